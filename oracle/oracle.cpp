// FP64 CPU oracle for spherical-cap GGX VNDF sampling (Dupuy & Benyoub,
// "Sampling Visible GGX Normals with Spherical Caps", arXiv 2306.05044).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU library is checked against.  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it.  It shares no source,
// header, table or helper with the HIP library, and it never calls it.
//
// Every routine follows the paper's own statement of the mathematics, in the
// paper's order and notation, in double precision:
//   * Philox4x32-10 from its published definition (Salmon, Moraes, Dror,
//     Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4).
//   * the general VNDF sampler (Sec. 2, "Importance Sampling", steps 1-3)
//     wrapped around either hemisphere sampler:
//       - the spherical-cap sampler of Sec. 3.3 (cap in (-z_i, 1], then the
//         half vector, normalised only after the unstretch), or
//       - Heitz's 2018 cross-section sampler of Sec. 2 (comparison baseline);
//   * the VNDF pdf as a linearly transformed hemisphere VNDF, Eqs. (1)-(4);
//   * the GGX NDF, Smith G1/G2 and Cook-Torrance BRDF of Appendix A;
//   * the Monte Carlo estimator of the direct-illumination integral,
//     Appendix A, "Importance Sampling Using the GGX VNDF", with L == 1
//     (directional albedo), weight f_r |cos theta_b| / PDF evaluated
//     literally (no algebraic simplification);
//   * its gradient by forward-mode dual numbers (exact derivative of this
//     same program) and by central finite differences;
//   * the same estimator with a non-constant incident radiance (a sum of
//     spherical-Gaussian lobes), i.e. the direct-illumination integral;
//   * a rough dielectric (reflection and transmission) sampled with the same
//     VNDF, after Walter et al. 2007, whom the paper cites for it: Fresnel
//     equations, Snell's law, generalised half vector and its Jacobian.
//
// Readings where the paper is silent:
//   * u1 drives the azimuth and u2 the height, exactly as the cap listing.
//   * Random numbers: u = (w >> 8) * 2^-24 from Philox words; counter
//     (lo32(k>>1), unit, tag, hi32(k>>1)), key (lo32(seed), hi32(seed));
//     sample k takes words (w0, w1) if k is even, else (w2, w3).
//   * G1 is zero when the direction lies at or below the horizon (the
//     printed G1 lacks that factor), so the pdf is zero there too.
//   * Fresnel is Schlick's: F0 + (1 - F0)(1 - x)^5 with x = wh . wo.
//   * Reflected directions at or below the horizon carry zero weight but
//     still count in N.
//   * Inputs outside the domain (w_z <= 0, alpha <= 0) give h = (0,0,1)
//     and pdf = 0; albedo cells with wo_z <= 0 give 0 and zero gradient.
//   * Dielectric: eta = n_lower / n_upper with wi above; lobe chosen by a third
//     uniform u3 < F (reflect); uniforms from one Philox block per sample
//     (counter (lo32(k), unit, 5, hi32(k)), words 0..2); the transmission G2
//     is the same height-correlated combination as for reflection.
//   * grad_theta_o is the derivative along the meridian of wo at fixed
//     azimuth: dwo/dtheta = (cos t cos p, cos t sin p, -sin t); at the pole
//     the azimuth is taken as 0.
//
// Precision: double, except where double is not enough for the tolerance the
// oracle checks.  A sampled normal near the rim of the cap, seen from the
// side opposite to wi, is the half vector of two nearly opposite unit
// vectors: forming it literally loses 2^-53 times the conditioning
// kappa = max(1, ax, ay) / |M^-T (c + wi_std)| (up to 2^24 for 24-bit
// uniforms), and the pdf of Eq. (1) at that normal is as sensitive.  The
// sampler therefore evaluates every tuple in double, and again, with the same
// code, in quadruple precision (__float128) when the double result has
// kappa > 1e4; the outputs are the double roundings of that evaluation.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <quadmath.h>

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (SC'11, Sec. 4): a 10-round Feistel-like network.  Each round
// multiplies words 0 and 2 by the two round constants into 64-bit products;
// the new words are (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
// lo(M0*c0)).  The key is bumped by the two Weyl constants between rounds.
// ---------------------------------------------------------------------------
const uint32_t kPhiloxM0 = 0xD2511F53u;
const uint32_t kPhiloxM1 = 0xCD9E8D57u;
const uint32_t kPhiloxW0 = 0x9E3779B9u;
const uint32_t kPhiloxW1 = 0xBB67AE85u;

void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {in[0], in[1], in[2], in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += kPhiloxW0;
            k[1] += kPhiloxW1;
        }
        uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// 24-bit uniform in [0, 1): top 24 bits of the word times 2^-24.
double word_to_unit(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

// The two uniforms of sample k of stream (seed, tag, unit).
void stream_uniforms(uint64_t seed, uint32_t tag, uint32_t unit, uint64_t k,
                     double* u1, double* u2) {
    uint64_t pair = k >> 1;
    uint32_t ctr[4] = {(uint32_t)pair, unit, tag, (uint32_t)(pair >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    if ((k & 1u) == 0) {
        *u1 = word_to_unit(w[0]);
        *u2 = word_to_unit(w[1]);
    } else {
        *u1 = word_to_unit(w[2]);
        *u2 = word_to_unit(w[3]);
    }
}

const uint32_t kTagSample = 2;  // vndf_sample tuples, unit 0, k = tuple index
const uint32_t kTagAlbedo = 3;  // estimator samples, unit = cell / job index

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with three tangents (alpha_x, alpha_y, theta_o).
// ---------------------------------------------------------------------------
struct Dual3 {
    double v;
    double d[3];
    Dual3() : v(0.0), d{0.0, 0.0, 0.0} {}
    Dual3(double x) : v(x), d{0.0, 0.0, 0.0} {}  // NOLINT: implicit by design
    Dual3(double x, double d0, double d1, double d2) : v(x), d{d0, d1, d2} {}
};
inline Dual3 operator+(const Dual3& a, const Dual3& b) {
    return Dual3(a.v + b.v, a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]);
}
inline Dual3 operator-(const Dual3& a, const Dual3& b) {
    return Dual3(a.v - b.v, a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]);
}
inline Dual3 operator-(const Dual3& a) { return Dual3(-a.v, -a.d[0], -a.d[1], -a.d[2]); }
inline Dual3 operator*(const Dual3& a, const Dual3& b) {
    return Dual3(a.v * b.v, a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1],
                 a.d[2] * b.v + a.v * b.d[2]);
}
inline Dual3 operator/(const Dual3& a, const Dual3& b) {
    double q = a.v / b.v;
    return Dual3(q, (a.d[0] - q * b.d[0]) / b.v, (a.d[1] - q * b.d[1]) / b.v,
                 (a.d[2] - q * b.d[2]) / b.v);
}
inline Dual3 sqrt(const Dual3& a) {
    double s = std::sqrt(a.v);
    // At an argument of exactly zero the only way here is the clamp of a
    // quantity that is identically zero (u2 == 0 puts the sample at the apex
    // of the cap for every parameter value), so its derivative is zero.
    if (s == 0.0) return Dual3(0.0);
    double f = 0.5 / s;
    return Dual3(s, a.d[0] * f, a.d[1] * f, a.d[2] * f);
}
inline double value(double x) { return x; }
inline double value(const Dual3& x) { return x.v; }
inline double sqrt_(double x) { return std::sqrt(x); }

// Quadruple precision for the ill-conditioned samples of the sampler.
using Quad = __float128;
inline double value(Quad x) { return (double)x; }
inline Quad sqrt_(Quad x) { return sqrtq(x); }
// The scalar type of a sampler's constants: double, except under Quad.
template <class T> struct ScalarOf { using type = double; };
template <> struct ScalarOf<Quad> { using type = Quad; };
inline double cos_(double x) { return std::cos(x); }
inline double sin_(double x) { return std::sin(x); }
inline Quad cos_(Quad x) { return cosq(x); }
inline Quad sin_(Quad x) { return sinq(x); }
template <class S> S pi_of();
template <> inline double pi_of<double>() { return kPi; }
template <> inline Quad pi_of<Quad>() { return M_PIq; }
inline Dual3 sqrt_(const Dual3& x) { return sqrt(x); }

template <class T>
struct Vec3 {
    T x, y, z;
};
template <class T>
T dot(const Vec3<T>& a, const Vec3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
Vec3<T> normalize(const Vec3<T>& a) {
    T n = sqrt_(dot(a, a));
    return Vec3<T>{a.x / n, a.y / n, a.z / n};
}
template <class T>
Vec3<T> cross(const Vec3<T>& a, const Vec3<T>& b) {
    return Vec3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T>
T clamp01(const T& x) {
    if (value(x) < 0.0) return T(0.0);
    if (value(x) > 1.0) return T(1.0);
    return x;
}
template <class T>
T max0(const T& x) { return value(x) > 0.0 ? x : T(0.0); }

// ---------------------------------------------------------------------------
// Hemisphere samplers (the visible normals of the unit hemisphere seen from
// direction wi, which is unit and above the horizon).
// ---------------------------------------------------------------------------

// Spherical-cap sampler, Sec. 3.2-3.3.  The visible normals of the
// hemisphere seen from wi are the half vectors between wi and directions c
// drawn uniformly on the part of the unit sphere with c_z > -wi_z (the
// directions whose half vector with wi lies in the upper hemisphere).  By
// Archimedes' hat-box theorem the zone of the unit sphere above height t has
// area 2 pi (1 - t), so a uniform point of that cap has a uniform height:
// P(c_z >= t) = (1 - t) / (1 + wi_z) on (-wi_z, 1]; its azimuth is uniform.
// u2 selects the height (u2 = 0 at the apex), u1 the azimuth.  Returns
// wi + c without normalising it.
template <class T>
Vec3<T> hemisphere_cap(double u1, double u2, const Vec3<T>& wi) {
    using S = typename ScalarOf<T>::type;
    const T height = T(1.0) - S(u2) * (T(1.0) + wi.z);
    const T radius = sqrt_(clamp01(T(1.0) - height * height));
    const S azimuth = S(2.0) * pi_of<S>() * S(u1);
    const Vec3<T> c{radius * cos_(azimuth), radius * sin_(azimuth), height};
    return Vec3<T>{wi.x + c.x, wi.y + c.y, wi.z + c.z};
}

// Heitz's cross-section sampler (JCGT 7(4), 2018; the paper's Sec. 2
// baseline).  Seen from wi, the visible hemisphere projects onto the plane
// orthogonal to wi as half of the unit disk joined to half of an ellipse
// whose short axis is wi_z; its visible normals are the points of that
// projected area, drawn uniformly, lifted back onto the hemisphere.  A
// uniform point of the unit disk (radius sqrt(u2), azimuth 2 pi u1: the same
// roles as the cap's) is mapped onto the projected area by moving its second
// coordinate, along lines of constant first coordinate, from the full
// disk's chord onto the chord of the half disk + half ellipse: with
// s = (1 + wi_z) / 2 (the fraction of the projected area on the disk side),
// d2 -> (1 - s) sqrt(1 - d1^2) + s d2.
template <class T>
Vec3<T> hemisphere_disk2018(double u1, double u2, const Vec3<T>& wi) {
    // frame (e1, e2, wi): e1 horizontal and orthogonal to wi
    const T horiz = wi.x * wi.x + wi.y * wi.y;
    Vec3<T> e1{T(1.0), T(0.0), T(0.0)};
    if (value(horiz) > 0.0) {
        const T inv = T(1.0) / sqrt_(horiz);
        e1 = Vec3<T>{-wi.y * inv, wi.x * inv, T(0.0)};
    }
    const Vec3<T> e2 = cross(wi, e1);
    // uniform point of the unit disk
    using S = typename ScalarOf<T>::type;
    const S rad = sqrt_(S(u2)), ang = S(2.0) * pi_of<S>() * S(u1);
    const T d1 = T(rad * cos_(ang));
    T d2 = T(rad * sin_(ang));
    // onto the projected visible area
    const T frac_disk = (T(1.0) + wi.z) / 2.0;
    d2 = frac_disk * d2 + (T(1.0) - frac_disk) * sqrt_(T(1.0) - d1 * d1);
    // lift onto the hemisphere: the normal's component along wi
    const T lift = sqrt_(max0(T(1.0) - d1 * d1 - d2 * d2));
    return Vec3<T>{d1 * e1.x + d2 * e2.x + lift * wi.x, d1 * e1.y + d2 * e2.y + lift * wi.y,
                   d1 * e1.z + d2 * e2.z + lift * wi.z};
}

// General VNDF sampler (Sec. 2, "Importance Sampling"): warp wi by M^-1 =
// diag(ax, ay, 1) and normalise, sample the hemisphere, warp the normal back
// with M^-T = diag(ax, ay, 1) and normalise.
template <class T>
Vec3<T> sample_vndf(double u1, double u2, const Vec3<T>& wi, const T& ax, const T& ay,
                    int method) {
    Vec3<T> wi_std = normalize(Vec3<T>{wi.x * ax, wi.y * ay, wi.z});
    Vec3<T> wm_std = method == 0 ? hemisphere_cap(u1, u2, wi_std)
                                 : hemisphere_disk2018(u1, u2, wi_std);
    return normalize(Vec3<T>{wm_std.x * ax, wm_std.y * ay, wm_std.z});
}

// ---------------------------------------------------------------------------
// Densities.
// ---------------------------------------------------------------------------

// Hemisphere NDF, Eq. (3): 1/pi above the horizon.
template <class T>
T ndf_std(const Vec3<T>& wm) {
    using S = typename ScalarOf<T>::type;
    return value(wm.z) > 0.0 ? T(S(1.0) / pi_of<S>()) : T(0.0);
}

// Cross-sectional area of the hemisphere seen from wi, Eq. (4).
template <class T>
T sigma_std(const Vec3<T>& wi) { return (T(1.0) + wi.z) / 2.0; }

// Hemisphere VNDF, Eq. (2).
template <class T>
T vndf_std(const Vec3<T>& wm, const Vec3<T>& wi) {
    return max0(dot(wm, wi)) * ndf_std(wm) / sigma_std(wi);
}

// GGX VNDF as a linearly transformed hemisphere VNDF, Eq. (1): the
// hemisphere VNDF of M^T wm / |M^T wm| seen from M^-1 wi / |M^-1 wi|, times
// the Jacobian |det M^T| / |M^T wm|^3, with M = diag(1/ax, 1/ay, 1).
template <class T>
T vndf_pdf(const Vec3<T>& wm, const Vec3<T>& wi, T ax, T ay) {
    if (!(value(wi.z) > 0.0) || !(value(ax) > 0.0) || !(value(ay) > 0.0)) return T(0.0);
    Vec3<T> mtwm{wm.x / ax, wm.y / ay, wm.z};
    T len = sqrt_(dot(mtwm, mtwm));
    Vec3<T> wm_std{mtwm.x / len, mtwm.y / len, mtwm.z / len};
    Vec3<T> wi_std = normalize(Vec3<T>{wi.x * ax, wi.y * ay, wi.z});
    T det = T(1.0) / (ax * ay);
    return vndf_std(wm_std, wi_std) * det / (len * len * len);
}

// Conditioning of a cap sample (see the header): max(1, ax, ay) / L with
// L = |M^-T hs| and |hs| = 2 wi_std . h_std, from the sampled normal h.
double cap_conditioning(const Vec3<double>& h, const Vec3<double>& wi, double ax, double ay) {
    Vec3<double> mth{h.x / ax, h.y / ay, h.z};
    double len = std::sqrt(dot(mth, mth));
    Vec3<double> wi_std = normalize(Vec3<double>{wi.x * ax, wi.y * ay, wi.z});
    double hs = 2.0 * dot(mth, wi_std) / len;
    if (!(hs > 0.0)) return HUGE_VAL;
    return std::max(1.0, std::max(ax, ay)) * len / hs;
}

const double kQuadKappa = 1e4;

// GGX NDF, Appendix A: the hemisphere NDF of M^T wm / |M^T wm| times the
// Jacobian |det M^T| / |M^T wm|^4.
template <class T>
T ggx_ndf(const Vec3<T>& wm, const T& ax, const T& ay) {
    Vec3<T> mtwm{wm.x / ax, wm.y / ay, wm.z};
    T len = sqrt_(dot(mtwm, mtwm));
    Vec3<T> wm_std{mtwm.x / len, mtwm.y / len, mtwm.z / len};
    T det = T(1.0) / (ax * ay);
    T len2 = len * len;
    return ndf_std(wm_std) * det / (len2 * len2);
}

// Smith monostatic shadowing G1(wm, wk), Appendix A, in its hemisphere form:
// chi+(wk_std . wm_std) z_k_std / sigma_std(wk_std).  Zero at or below the
// horizon (reading of the printed formula, which lacks that factor).
template <class T>
T smith_g1(const Vec3<T>& wm, const Vec3<T>& wk, const T& ax, const T& ay) {
    if (!(value(wk.z) > 0.0)) return T(0.0);
    Vec3<T> wm_std = normalize(Vec3<T>{wm.x / ax, wm.y / ay, wm.z});
    Vec3<T> wk_std = normalize(Vec3<T>{wk.x * ax, wk.y * ay, wk.z});
    if (!(value(dot(wk_std, wm_std)) > 0.0)) return T(0.0);
    return wk_std.z / sigma_std(wk_std);
}

// Height-correlated Smith G2, Appendix A.
template <class T>
T smith_g2(const Vec3<T>& wm, const Vec3<T>& wi, const Vec3<T>& wo, const T& ax,
           const T& ay) {
    T gi = smith_g1(wm, wi, ax, ay);
    T go = smith_g1(wm, wo, ax, ay);
    T den = gi + go - gi * go;
    if (!(value(den) > 0.0)) return T(0.0);
    return gi * go / den;
}

// Schlick's Fresnel (the paper names F without a formula).
template <class T>
T fresnel_schlick(const T& x, double f0) {
    T m = T(1.0) - x;
    T m2 = m * m;
    return f0 + (1.0 - f0) * (m2 * m2 * m);
}

// Cook-Torrance BRDF, Appendix A: F(wh . wo) G2 D / (4 cos(theta_i) cos(theta_o)),
// here with wi = the view direction wa and wo = the generated direction wb.
template <class T>
T brdf_ggx(const Vec3<T>& wa, const Vec3<T>& wb, const T& ax, const T& ay, double f0) {
    if (!(value(wa.z) > 0.0) || !(value(wb.z) > 0.0)) return T(0.0);
    Vec3<T> wh = normalize(Vec3<T>{wa.x + wb.x, wa.y + wb.y, wa.z + wb.z});
    T f = fresnel_schlick(dot(wh, wb), f0);
    T g2 = smith_g2(wh, wa, wb, ax, ay);
    T d = ggx_ndf(wh, ax, ay);
    return f * g2 * d / (4.0 * wa.z * wb.z);
}

// One term of the albedo estimator (Appendix A, "Importance Sampling Using the
// GGX VNDF", L == 1): sample wm from the VNDF seen from wa, reflect wa about
// it, and return f_r(wb, wa) |cos theta_b| / PDF(wb, wa) with
// PDF = G1(wm, wa) D(wm) / (4 cos theta_a).
template <class T>
T albedo_term(const Vec3<T>& wa, const T& ax, const T& ay, double u1, double u2, double f0,
              int method) {
    Vec3<T> wm = sample_vndf(u1, u2, wa, ax, ay, method);
    T c = dot(wm, wa);
    Vec3<T> wb{2.0 * c * wm.x - wa.x, 2.0 * c * wm.y - wa.y, 2.0 * c * wm.z - wa.z};
    if (!(value(wb.z) > 0.0)) return T(0.0);
    T fr = brdf_ggx(wa, wb, ax, ay, f0);
    T cos_b = wb.z;
    T pdf = smith_g1(wm, wa, ax, ay) * ggx_ndf(wm, ax, ay) / (4.0 * wa.z);
    if (!(value(pdf) > 0.0)) return T(0.0);
    return fr * cos_b / pdf;
}

// Neumaier (Kahan-Babuska) compensated sum.
template <class T>
struct NeumaierSum {
    T s, c;
    NeumaierSum() : s(0.0), c(0.0) {}
    void add(const T& x) {
        T t = s + x;
        if (std::fabs(value(s)) >= std::fabs(value(x)))
            c = c + ((s - t) + x);
        else
            c = c + ((x - t) + s);
        s = t;
    }
    T result() const { return s + c; }
};

// Run body(i) for i in [0, n) over nthreads threads (static contiguous split).
template <class F>
void parallel_for(int64_t n, int nthreads, F body) {
    if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
    if (n <= 0) return;
    if (nthreads > n) nthreads = (int)n;
    if (nthreads == 1) {
        for (int64_t i = 0; i < n; ++i) body(i);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
        pool.emplace_back([=]() {
            for (int64_t i = lo; i < hi; ++i) body(i);
        });
    }
    for (auto& th : pool) th.join();
}

Vec3<double> unit_view(double x, double y, double z) {
    double n = std::sqrt(x * x + y * y + z * z);
    return Vec3<double>{x / n, y / n, z / n};
}

// Meridian tangent dwo/dtheta of a unit wo (azimuth 0 at the pole).
Vec3<double> meridian_tangent(const Vec3<double>& wo) {
    double rho = std::sqrt(wo.x * wo.x + wo.y * wo.y);
    if (rho > 0.0) return Vec3<double>{wo.z * wo.x / rho, wo.z * wo.y / rho, -rho};
    return Vec3<double>{wo.z, 0.0, 0.0};
}

double cell_albedo(const Vec3<double>& wo, double ax, double ay, int64_t n, uint64_t seed,
                   uint32_t unit, double f0, int method) {
    if (n <= 0 || !(wo.z > 0.0) || !(ax > 0.0) || !(ay > 0.0)) return 0.0;
    NeumaierSum<double> acc;
    for (int64_t k = 0; k < n; ++k) {
        double u1, u2;
        stream_uniforms(seed, kTagAlbedo, unit, (uint64_t)k, &u1, &u2);
        acc.add(albedo_term(wo, ax, ay, u1, u2, f0, method));
    }
    return acc.result() / (double)n;
}

// Synthetic incident radiance: a sum of spherical-Gaussian lobes,
// L(w) = sum_k lambda_k exp(kappa_k (mu_k . w - 1)) for unit w (a lobe with
// kappa = 0 is a constant term).  Lobe k is params[5k .. 5k+4] =
// (mu_x, mu_y, mu_z, kappa, lambda) with mu unit.
double radiance(const Vec3<double>& w, const double* params, int nlobes) {
    double l = 0.0;
    for (int k = 0; k < nlobes; ++k) {
        const double* p = params + 5 * k;
        const double c = p[0] * w.x + p[1] * w.y + p[2] * w.z;
        l += p[4] * std::exp(p[3] * (c - 1.0));
    }
    return l;
}

// One term of the direct-illumination estimator (Appendix A): sample wm from
// the VNDF seen from wa, reflect, and return L(wb) f_r(wb, wa) |cos theta_b| /
// PDF(wb, wa).
double radiance_term(const Vec3<double>& wa, double ax, double ay, double u1, double u2,
                     double f0, const double* params, int nlobes) {
    Vec3<double> wm = sample_vndf(u1, u2, wa, ax, ay, 0);
    double c = dot(wm, wa);
    Vec3<double> wb{2.0 * c * wm.x - wa.x, 2.0 * c * wm.y - wa.y, 2.0 * c * wm.z - wa.z};
    if (!(wb.z > 0.0)) return 0.0;
    double fr = brdf_ggx(wa, wb, ax, ay, f0);
    double pdf = smith_g1(wm, wa, ax, ay) * ggx_ndf(wm, ax, ay) / (4.0 * wa.z);
    if (!(pdf > 0.0)) return 0.0;
    return radiance(normalize(wb), params, nlobes) * fr * wb.z / pdf;
}


// ---------------------------------------------------------------------------
// Rough dielectric interface (reflection and transmission) sampled with the
// same VNDF.  The paper applies its sampler to rough dielectrics but states
// the transmission model only by reference to Walter, Marschner, Li and
// Torrance, "Microfacet models for refraction through rough surfaces"
// (EGSR 2007); the routines below follow that paper's definitions, in its
// notation, with wi on the upper side (index of refraction 1) and eta the
// relative index n_lower / n_upper.
// ---------------------------------------------------------------------------

const uint32_t kTagDielectric = 5;  // dielectric_sample tuples, unit 0, k = tuple index

// The three uniforms of sample k of the dielectric stream: one Philox block
// per sample, counter (lo32(k), unit, tag, hi32(k)), words 0, 1, 2.
void dielectric_uniforms(uint64_t seed, uint32_t unit, uint64_t k, double* u1, double* u2,
                         double* u3) {
    uint32_t ctr[4] = {(uint32_t)k, unit, kTagDielectric, (uint32_t)(k >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    *u1 = word_to_unit(w[0]);
    *u2 = word_to_unit(w[1]);
    *u3 = word_to_unit(w[2]);
}

// Unpolarised Fresnel reflectance of a smooth dielectric interface (the
// Fresnel equations): light arrives at cosine cos_i > 0 from the side of
// index n_i and refracts into index n_t, eta = n_t / n_i.  The s- and
// p-polarised amplitude ratios are
//   r_s = (n_i cos_i - n_t cos_t) / (n_i cos_i + n_t cos_t),
//   r_p = (n_t cos_i - n_i cos_t) / (n_t cos_i + n_i cos_t),
// with Snell's law n_i sin_i = n_t sin_t; R = (r_s^2 + r_p^2) / 2, and R = 1
// under total internal reflection.
double fresnel_dielectric(double cos_i, double eta) {
    double sin_i2 = std::max(0.0, 1.0 - cos_i * cos_i);
    double sin_t2 = sin_i2 / (eta * eta);
    if (sin_t2 >= 1.0) return 1.0;
    double cos_t = std::sqrt(1.0 - sin_t2);
    double rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);
    double rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);
    return 0.5 * (rs * rs + rp * rp);
}

// Smith G1 for a direction on either side of the surface (Walter et al.,
// Eq. (23) for GGX): chi+((v . m) / (v . n)) times the monostatic term of the
// unsigned direction, written here in the paper's hemisphere form
// z_std / sigma_std of the flipped-up direction.
double smith_g1_two_sided(const Vec3<double>& wm, const Vec3<double>& v, double ax, double ay) {
    if (v.z == 0.0) return 0.0;
    if (!(dot(v, wm) / v.z > 0.0)) return 0.0;
    Vec3<double> up = v.z > 0.0 ? v : Vec3<double>{-v.x, -v.y, -v.z};
    Vec3<double> up_std = normalize(Vec3<double>{up.x * ax, up.y * ay, up.z});
    return up_std.z / sigma_std(up_std);
}

// Height-correlated G2 built from the two one-sided terms, as in the
// paper's Appendix A (the same combination for both lobes).
double smith_g2_two_sided(const Vec3<double>& wm, const Vec3<double>& wi, const Vec3<double>& wo,
                          double ax, double ay) {
    double gi = smith_g1_two_sided(wm, wi, ax, ay);
    double go = smith_g1_two_sided(wm, wo, ax, ay);
    double den = gi + go - gi * go;
    if (!(den > 0.0)) return 0.0;
    return gi * go / den;
}

// Half vector of a pair (wi, wo): h_r = wi + wo for reflection (wo above the
// surface), the generalised h_t = -(wi + eta wo) for transmission (Walter et
// al., Eqs. (13) and (16)); normalised and turned to the upper side.
Vec3<double> dielectric_half(const Vec3<double>& wi, const Vec3<double>& wo, double eta) {
    Vec3<double> h = wo.z > 0.0 ? Vec3<double>{wi.x + wo.x, wi.y + wo.y, wi.z + wo.z}
                                : Vec3<double>{-(wi.x + eta * wo.x), -(wi.y + eta * wo.y),
                                               -(wi.z + eta * wo.z)};
    h = normalize(h);
    if (h.z < 0.0) h = Vec3<double>{-h.x, -h.y, -h.z};
    return h;
}

// BSDF of the rough dielectric (Walter et al., Eqs. (20) and (21)), radiance
// scaling by eta^2 included in the transmission term as printed there:
//   f_r = F G2 D / (4 |wi.n| |wo.n|),
//   f_t = |wi.h| |wo.h| / (|wi.n| |wo.n|) * eta^2 (1 - F) G2 D / (wi.h + eta wo.h)^2.
double dielectric_bsdf(const Vec3<double>& wi, const Vec3<double>& wo, double ax, double ay,
                       double eta) {
    if (!(wi.z > 0.0) || wo.z == 0.0) return 0.0;
    Vec3<double> h = dielectric_half(wi, wo, eta);
    double ci = dot(wi, h), co = dot(wo, h);
    if (!(ci > 0.0)) return 0.0;
    double f = fresnel_dielectric(ci, eta);
    double g2 = smith_g2_two_sided(h, wi, wo, ax, ay);
    double d = ggx_ndf(h, ax, ay);
    if (wo.z > 0.0) return f * g2 * d / (4.0 * wi.z * wo.z);
    if (!(co < 0.0)) return 0.0;
    double den = ci + eta * co;
    return std::fabs(ci) * std::fabs(co) / (wi.z * std::fabs(wo.z)) * eta * eta * (1.0 - f) *
           g2 * d / (den * den);
}

// Density of the dielectric sampler at wo (solid angle): the lobe's selection
// probability (F or 1 - F) times the VNDF of Eq. (1) at the half vector times
// the Jacobian |dh/dwo| of Walter et al., Eqs. (14) and (17):
//   reflection 1 / (4 |wo.h|),  transmission eta^2 |wo.h| / (wi.h + eta wo.h)^2.
double dielectric_pdf(const Vec3<double>& wi, const Vec3<double>& wo, double ax, double ay,
                      double eta) {
    if (!(wi.z > 0.0) || !(ax > 0.0) || !(ay > 0.0) || wo.z == 0.0) return 0.0;
    Vec3<double> h = dielectric_half(wi, wo, eta);
    double ci = dot(wi, h), co = dot(wo, h);
    if (!(ci > 0.0)) return 0.0;
    double f = fresnel_dielectric(ci, eta);
    double dv = vndf_pdf(h, wi, ax, ay);
    if (wo.z > 0.0) return f * dv / (4.0 * std::fabs(co));
    if (!(co < 0.0)) return 0.0;
    double den = ci + eta * co;
    return (1.0 - f) * dv * eta * eta * std::fabs(co) / (den * den);
}

struct DielectricSample {
    Vec3<double> h, wo;
    double pdf, weight;
    int lobe;  // 0 reflection, 1 transmission
};

// The sampler: a visible normal h from the spherical-cap VNDF sampler, the
// lobe from u3 against the Fresnel reflectance at wi . h (reflect if u3 < F),
// then the mirror direction 2 (wi.h) h - wi or the refracted direction of
// Snell's law in vector form (Walter et al., Eq. (40)),
//   wo = (c / eta - sqrt(1 - (1 - c^2) / eta^2)) h - wi / eta,  c = wi . h.
// A direction on the wrong side of the surface for its lobe is no sample
// (pdf 0, weight 0).  weight = f |wo.n| / pdf.
DielectricSample dielectric_sample(double u1, double u2, double u3, const Vec3<double>& wi,
                                   double ax, double ay, double eta) {
    DielectricSample s;
    s.h = sample_vndf(u1, u2, wi, ax, ay, 0);
    double c = dot(wi, s.h);
    double f = fresnel_dielectric(c, eta);
    bool valid;
    if (u3 < f) {
        s.lobe = 0;
        s.wo = Vec3<double>{2.0 * c * s.h.x - wi.x, 2.0 * c * s.h.y - wi.y, 2.0 * c * s.h.z - wi.z};
        valid = s.wo.z > 0.0;
    } else {
        s.lobe = 1;
        double k = std::sqrt(1.0 - (1.0 - c * c) / (eta * eta));
        double a = c / eta - k;
        s.wo = Vec3<double>{a * s.h.x - wi.x / eta, a * s.h.y - wi.y / eta, a * s.h.z - wi.z / eta};
        valid = s.wo.z < 0.0;
    }
    s.pdf = 0.0;
    s.weight = 0.0;
    if (valid) {
        s.pdf = dielectric_pdf(wi, s.wo, ax, ay, eta);
        if (s.pdf > 0.0) s.weight = dielectric_bsdf(wi, s.wo, ax, ay, eta) * std::fabs(s.wo.z) / s.pdf;
    }
    return s;
}

}  // namespace

extern "C" {

// Raw Philox4x32-10 block: out = philox(ctr, key).
void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
}

// Uniforms of samples k0 .. k0+n-1 of stream (seed, tag, unit).
void orc_uniforms(uint64_t seed, uint32_t tag, uint32_t unit, uint64_t k0, int64_t n,
                  double* u1, double* u2) {
    for (int64_t i = 0; i < n; ++i) stream_uniforms(seed, tag, unit, k0 + (uint64_t)i, &u1[i], &u2[i]);
}

// Hemisphere sampler alone (unit, upper-hemisphere wi): the raw unnormalised
// output of the chosen hemisphere routine.
void orc_hemisphere_sample(int64_t n, const double* wix, const double* wiy, const double* wiz,
                           const double* u1, const double* u2, int32_t method, double* hx,
                           double* hy, double* hz) {
    for (int64_t i = 0; i < n; ++i) {
        Vec3<double> wi{wix[i], wiy[i], wiz[i]};
        Vec3<double> h = method == 0 ? hemisphere_cap(u1[i], u2[i], wi)
                                     : hemisphere_disk2018(u1[i], u2[i], wi);
        hx[i] = h.x; hy[i] = h.y; hz[i] = h.z;
    }
}

// GGX VNDF sampling of n tuples.  u1/u2 both null: Philox stream
// (seed, tag 2, unit 0) at sample index index_base + i.  pdf may be null; it
// is the VNDF pdf of Eq. (1) evaluated at the sample.
int32_t orc_vndf_sample(int64_t n, const double* wix, const double* wiy, const double* wiz,
                        const double* ax, const double* ay, const double* u1, const double* u2,
                        uint64_t seed, uint64_t index_base, int32_t method, double* hx,
                        double* hy, double* hz, double* pdf, int32_t nthreads) {
    if (n < 0 || (method != 0 && method != 1)) return -1;
    if ((u1 == nullptr) != (u2 == nullptr)) return -1;
    parallel_for(n, nthreads, [&](int64_t i) {
        Vec3<double> wi{wix[i], wiy[i], wiz[i]};
        double a = ax[i], b = ay[i];
        double r1, r2;
        if (u1 != nullptr) {
            r1 = u1[i]; r2 = u2[i];
        } else {
            stream_uniforms(seed, kTagSample, 0u, index_base + (uint64_t)i, &r1, &r2);
        }
        if (!(wi.z > 0.0) || !(a > 0.0) || !(b > 0.0)) {
            hx[i] = 0.0; hy[i] = 0.0; hz[i] = 1.0;
            if (pdf) pdf[i] = 0.0;
            return;
        }
        Vec3<double> h = sample_vndf(r1, r2, wi, a, b, method);
        double p = pdf ? vndf_pdf(h, wi, a, b) : 0.0;
        if (cap_conditioning(h, wi, a, b) > kQuadKappa) {
            const Vec3<Quad> wq{(Quad)wi.x, (Quad)wi.y, (Quad)wi.z};
            const Vec3<Quad> hq = sample_vndf(r1, r2, wq, (Quad)a, (Quad)b, method);
            h = Vec3<double>{(double)hq.x, (double)hq.y, (double)hq.z};
            if (pdf) p = (double)vndf_pdf(hq, wq, (Quad)a, (Quad)b);
        }
        hx[i] = h.x; hy[i] = h.y; hz[i] = h.z;
        if (pdf) pdf[i] = p;
    });
    return 0;
}

// VNDF pdf of Eq. (1) at caller-given (wm, wi, alpha).
int32_t orc_vndf_pdf(int64_t n, const double* wix, const double* wiy, const double* wiz,
                     const double* hx, const double* hy, const double* hz, const double* ax,
                     const double* ay, double* pdf, int32_t nthreads) {
    if (n < 0) return -1;
    parallel_for(n, nthreads, [&](int64_t i) {
        pdf[i] = vndf_pdf(Vec3<double>{hx[i], hy[i], hz[i]}, Vec3<double>{wix[i], wiy[i], wiz[i]},
                          ax[i], ay[i]);
    });
    return 0;
}

// GGX NDF D(wm) and Smith G1(wm, wk) of Appendix A, element-wise.
void orc_ggx_ndf(int64_t n, const double* hx, const double* hy, const double* hz,
                 const double* ax, const double* ay, double* out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = ggx_ndf(Vec3<double>{hx[i], hy[i], hz[i]}, ax[i], ay[i]);
}
void orc_smith_g1(int64_t n, const double* hx, const double* hy, const double* hz,
                  const double* wx, const double* wy, const double* wz, const double* ax,
                  const double* ay, double* out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = smith_g1(Vec3<double>{hx[i], hy[i], hz[i]}, Vec3<double>{wx[i], wy[i], wz[i]},
                          ax[i], ay[i]);
}

// Cook-Torrance GGX BRDF f_r(wa, wb), element-wise (Appendix A).
void orc_brdf(int64_t n, const double* ax_, const double* ay_, const double* wax,
              const double* way, const double* waz, const double* wbx, const double* wby,
              const double* wbz, double f0, double* out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = brdf_ggx(Vec3<double>{wax[i], way[i], waz[i]}, Vec3<double>{wbx[i], wby[i], wbz[i]},
                          ax_[i], ay_[i], f0);
}

// Single estimator terms for caller-given uniforms (one per element).
void orc_albedo_terms(int64_t n, const double* wox, const double* woy, const double* woz,
                      const double* ax, const double* ay, const double* u1, const double* u2,
                      double f0, int32_t method, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        Vec3<double> wo{wox[i], woy[i], woz[i]};
        if (!(wo.z > 0.0) || !(ax[i] > 0.0) || !(ay[i] > 0.0)) { out[i] = 0.0; continue; }
        out[i] = albedo_term(unit_view(wo.x, wo.y, wo.z), ax[i], ay[i], u1[i], u2[i], f0, method);
    }
}

// Directional albedo per cell: (1/N) sum of the estimator terms over the
// Philox stream (seed, tag 3, unit = units[c] or c), Neumaier-summed.
int32_t orc_albedo(int64_t ncells, const double* wox, const double* woy, const double* woz,
                   const double* ax, const double* ay, const int64_t* nsamples,
                   const uint32_t* units, uint64_t seed, const double* f0, int32_t method,
                   double* albedo, int32_t nthreads) {
    if (ncells < 0) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        Vec3<double> wo = woz[c] > 0.0 ? unit_view(wox[c], woy[c], woz[c])
                                       : Vec3<double>{wox[c], woy[c], woz[c]};
        albedo[c] = cell_albedo(wo, ax[c], ay[c], nsamples[c], seed, unit, f0[c], method);
    });
    return 0;
}

// Albedo and its gradient w.r.t. (alpha_x, alpha_y, theta_o) per cell by
// forward-mode dual numbers through the same estimator (common random
// numbers: the gradient of this program's own output).
int32_t orc_albedo_grad(int64_t ncells, const double* wox, const double* woy, const double* woz,
                        const double* ax, const double* ay, const int64_t* nsamples,
                        const uint32_t* units, uint64_t seed, const double* f0, double* albedo,
                        double* g_ax, double* g_ay, double* g_theta, int32_t nthreads) {
    if (ncells < 0) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        int64_t n = nsamples[c];
        albedo[c] = 0.0; g_ax[c] = 0.0; g_ay[c] = 0.0; g_theta[c] = 0.0;
        if (n <= 0 || !(woz[c] > 0.0) || !(ax[c] > 0.0) || !(ay[c] > 0.0)) return;
        Vec3<double> wo = unit_view(wox[c], woy[c], woz[c]);
        Vec3<double> t = meridian_tangent(wo);
        Vec3<Dual3> wo_d{Dual3(wo.x, 0.0, 0.0, t.x), Dual3(wo.y, 0.0, 0.0, t.y),
                         Dual3(wo.z, 0.0, 0.0, t.z)};
        Dual3 a(ax[c], 1.0, 0.0, 0.0), b(ay[c], 0.0, 1.0, 0.0);
        NeumaierSum<double> sv, s0, s1, s2;
        for (int64_t k = 0; k < n; ++k) {
            double u1, u2;
            stream_uniforms(seed, kTagAlbedo, unit, (uint64_t)k, &u1, &u2);
            Dual3 w = albedo_term(wo_d, a, b, u1, u2, f0[c], 0);
            sv.add(w.v); s0.add(w.d[0]); s1.add(w.d[1]); s2.add(w.d[2]);
        }
        double inv = 1.0 / (double)n;
        albedo[c] = sv.result() * inv;
        g_ax[c] = s0.result() * inv;
        g_ay[c] = s1.result() * inv;
        g_theta[c] = s2.result() * inv;
    });
    return 0;
}

// Central finite differences of orc_albedo (same random numbers) with the
// given step for alpha_x, alpha_y and theta_o (wo moved along its meridian).
int32_t orc_albedo_fd(int64_t ncells, const double* wox, const double* woy, const double* woz,
                      const double* ax, const double* ay, const int64_t* nsamples,
                      const uint32_t* units, uint64_t seed, const double* f0, double step,
                      double* g_ax, double* g_ay, double* g_theta, int32_t nthreads) {
    if (ncells < 0 || !(step > 0.0)) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        int64_t n = nsamples[c];
        g_ax[c] = 0.0; g_ay[c] = 0.0; g_theta[c] = 0.0;
        if (n <= 0 || !(woz[c] > 0.0) || !(ax[c] > 0.0) || !(ay[c] > 0.0)) return;
        Vec3<double> wo = unit_view(wox[c], woy[c], woz[c]);
        double rho = std::sqrt(wo.x * wo.x + wo.y * wo.y);
        double theta = std::atan2(rho, wo.z);
        double phi = rho > 0.0 ? std::atan2(wo.y, wo.x) : 0.0;
        auto at = [&](double th) {
            return Vec3<double>{std::sin(th) * std::cos(phi), std::sin(th) * std::sin(phi),
                                std::cos(th)};
        };
        double a = ax[c], b = ay[c];
        g_ax[c] = (cell_albedo(wo, a + step, b, n, seed, unit, f0[c], 0) -
                   cell_albedo(wo, a - step, b, n, seed, unit, f0[c], 0)) / (2.0 * step);
        g_ay[c] = (cell_albedo(wo, a, b + step, n, seed, unit, f0[c], 0) -
                   cell_albedo(wo, a, b - step, n, seed, unit, f0[c], 0)) / (2.0 * step);
        g_theta[c] = (cell_albedo(at(theta + step), a, b, n, seed, unit, f0[c], 0) -
                      cell_albedo(at(theta - step), a, b, n, seed, unit, f0[c], 0)) / (2.0 * step);
    });
    return 0;
}

// Samples whose estimator term changes between zero and non-zero within a
// central-difference step (the reflection crosses the horizon there): per
// cell and parameter (alpha_x, alpha_y, theta_o) the number of samples k
// whose term at the parameter minus step, at it and at it plus step is zero
// at some of the three and non-zero at others.  There the term has a kink,
// so a central difference over the step does not approximate its slope.
int32_t orc_albedo_kinks(int64_t ncells, const double* wox, const double* woy, const double* woz,
                         const double* ax, const double* ay, const int64_t* nsamples,
                         const uint32_t* units, uint64_t seed, double step, int64_t* k_ax,
                         int64_t* k_ay, int64_t* k_theta, int32_t nthreads) {
    if (ncells < 0 || !(step > 0.0)) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        int64_t n = nsamples[c];
        k_ax[c] = 0; k_ay[c] = 0; k_theta[c] = 0;
        if (n <= 0 || !(woz[c] > 0.0) || !(ax[c] > 0.0) || !(ay[c] > 0.0)) return;
        Vec3<double> wo = unit_view(wox[c], woy[c], woz[c]);
        double rho = std::sqrt(wo.x * wo.x + wo.y * wo.y);
        double theta = std::atan2(rho, wo.z);
        double phi = rho > 0.0 ? std::atan2(wo.y, wo.x) : 0.0;
        auto at = [&](double th) {
            return Vec3<double>{std::sin(th) * std::cos(phi), std::sin(th) * std::sin(phi),
                                std::cos(th)};
        };
        const Vec3<double> wm = at(theta - step), wp = at(theta + step);
        double a = ax[c], b = ay[c];
        auto mixed = [](double x, double y, double z) {
            int live = (x != 0.0) + (y != 0.0) + (z != 0.0);
            return live != 0 && live != 3;
        };
        for (int64_t k = 0; k < n; ++k) {
            double u1, u2;
            stream_uniforms(seed, kTagAlbedo, unit, (uint64_t)k, &u1, &u2);
            double w0 = albedo_term(wo, a, b, u1, u2, 1.0, 0);
            k_ax[c] += mixed(albedo_term(wo, a - step, b, u1, u2, 1.0, 0), w0,
                             albedo_term(wo, a + step, b, u1, u2, 1.0, 0));
            k_ay[c] += mixed(albedo_term(wo, a, b - step, u1, u2, 1.0, 0), w0,
                             albedo_term(wo, a, b + step, u1, u2, 1.0, 0));
            k_theta[c] += mixed(albedo_term(wm, a, b, u1, u2, 1.0, 0), w0,
                                albedo_term(wp, a, b, u1, u2, 1.0, 0));
        }
    });
    return 0;
}

// Horizon band of an FP32 evaluation of the estimator.  A GPU sample whose
// reflected direction lies within its own rounding error of the horizon may
// land on the other side than the exact sample; its weight is continuous
// there but the weight's slope jumps from the live side's to 0.  Per cell,
// over the samples whose exact wb_z lies within (c0 + c1 kappa) 2^-24 of 0
// (kappa: the sample's conditioning, as for the sampler), this returns their
// count and (1/N) sum of |d/dp| of the live side's weight F G2 / G1(wa) for
// p = alpha_x, alpha_y, theta_o, with G1(wb) continued below the horizon by
// its hemisphere form 2 z / (1 + z) -- the most a change of side of those
// samples can move the gradient.  Samples with kappa > kappa_max are left
// out (the kernels evaluate those in double precision).
int32_t orc_albedo_horizon_band(int64_t ncells, const double* wox, const double* woy,
                                const double* woz, const double* ax, const double* ay,
                                const int64_t* nsamples, const uint32_t* units, uint64_t seed,
                                const double* f0, double c0, double c1, double kappa_max,
                                double* b_ax, double* b_ay, double* b_theta, int64_t* count,
                                int32_t nthreads) {
    if (ncells < 0) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        int64_t n = nsamples[c];
        b_ax[c] = 0.0; b_ay[c] = 0.0; b_theta[c] = 0.0; count[c] = 0;
        if (n <= 0 || !(woz[c] > 0.0) || !(ax[c] > 0.0) || !(ay[c] > 0.0)) return;
        Vec3<double> wo = unit_view(wox[c], woy[c], woz[c]);
        Vec3<double> t = meridian_tangent(wo);
        Vec3<Dual3> wo_d{Dual3(wo.x, 0.0, 0.0, t.x), Dual3(wo.y, 0.0, 0.0, t.y),
                         Dual3(wo.z, 0.0, 0.0, t.z)};
        Dual3 a(ax[c], 1.0, 0.0, 0.0), b(ay[c], 0.0, 1.0, 0.0);
        NeumaierSum<double> s0, s1, s2;
        for (int64_t k = 0; k < n; ++k) {
            double u1, u2;
            stream_uniforms(seed, kTagAlbedo, unit, (uint64_t)k, &u1, &u2);
            Vec3<double> wm = sample_vndf(u1, u2, wo, ax[c], ay[c], 0);
            double cm = dot(wm, wo);
            double wbz = 2.0 * cm * wm.z - wo.z;
            const double kap = cap_conditioning(wm, wo, ax[c], ay[c]);
            if (kap > kappa_max) continue;
            double band = (c0 + c1 * kap) * 0x1p-24;
            if (!(std::fabs(wbz) <= band)) continue;
            ++count[c];
            Vec3<Dual3> wmd = sample_vndf(u1, u2, wo_d, a, b, 0);
            Dual3 cd = dot(wmd, wo_d);
            Vec3<Dual3> wb{2.0 * cd * wmd.x - wo_d.x, 2.0 * cd * wmd.y - wo_d.y,
                           2.0 * cd * wmd.z - wo_d.z};
            Vec3<Dual3> wb_std = normalize(Vec3<Dual3>{wb.x * a, wb.y * b, wb.z});
            Dual3 gl = wb_std.z / sigma_std(wb_std);
            Dual3 go = smith_g1(wmd, wo_d, a, b);
            Dual3 g2 = go * gl / (go + gl - go * gl);
            Dual3 w = fresnel_schlick(cd, f0[c]) * g2 / go;
            s0.add(std::fabs(w.d[0])); s1.add(std::fabs(w.d[1])); s2.add(std::fabs(w.d[2]));
        }
        double inv = 1.0 / (double)n;
        b_ax[c] = s0.result() * inv;
        b_ay[c] = s1.result() * inv;
        b_theta[c] = s2.result() * inv;
    });
    return 0;
}

// Direct illumination per cell: (1/N) sum of radiance_term over the Philox
// stream (seed, tag 3, unit = units[c] or c), Neumaier-summed.
int32_t orc_radiance(int64_t ncells, const double* wox, const double* woy, const double* woz,
                     const double* ax, const double* ay, const double* f0,
                     const int64_t* nsamples, const uint32_t* units, uint64_t seed,
                     const double* lobes, int32_t nlobes, double* out, int32_t nthreads) {
    if (ncells < 0 || nlobes < 0) return -1;
    parallel_for(ncells, nthreads, [&](int64_t c) {
        uint32_t unit = units ? units[c] : (uint32_t)c;
        out[c] = 0.0;
        int64_t n = nsamples[c];
        if (n <= 0 || !(woz[c] > 0.0) || !(ax[c] > 0.0) || !(ay[c] > 0.0)) return;
        Vec3<double> wo = unit_view(wox[c], woy[c], woz[c]);
        NeumaierSum<double> acc;
        for (int64_t k = 0; k < n; ++k) {
            double u1, u2;
            stream_uniforms(seed, kTagAlbedo, unit, (uint64_t)k, &u1, &u2);
            acc.add(radiance_term(wo, ax[c], ay[c], u1, u2, f0[c], lobes, nlobes));
        }
        out[c] = acc.result() / (double)n;
    });
    return 0;
}

// The radiance L(w) of the lobe set at n unit directions.
void orc_radiance_at(int64_t n, const double* wx, const double* wy, const double* wz,
                     const double* lobes, int32_t nlobes, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = radiance(Vec3<double>{wx[i], wy[i], wz[i]}, lobes, nlobes);
}

// Inverse of the cap sampler (Sec. 3.2): from a normal h seen from wi, the
// hemisphere normal h_std = M^T h / |M^T h| reflects wi_std = M^-1 wi /
// |M^-1 wi| into the cap point c = 2 (h_std . wi_std) h_std - wi_std
// (reflection law); the cap's height z = (1 - u2)(1 + z_i) - z_i and azimuth
// 2 pi u1 then give (u1, u2).  Outside the domain (w_z <= 0, alpha <= 0,
// h_z <= 0 or wi . h <= 0) both outputs are -1.
int32_t orc_vndf_inverse(int64_t n, const double* wix, const double* wiy, const double* wiz,
                         const double* hx, const double* hy, const double* hz, const double* ax,
                         const double* ay, double* u1, double* u2, int32_t nthreads) {
    if (n < 0) return -1;
    parallel_for(n, nthreads, [&](int64_t i) {
        Vec3<double> wi{wix[i], wiy[i], wiz[i]};
        Vec3<double> h{hx[i], hy[i], hz[i]};
        double a = ax[i], b = ay[i];
        if (!(wi.z > 0.0) || !(a > 0.0) || !(b > 0.0) || !(h.z > 0.0) || !(dot(wi, h) > 0.0)) {
            u1[i] = -1.0; u2[i] = -1.0;
            return;
        }
        Vec3<double> h_std = normalize(Vec3<double>{h.x / a, h.y / b, h.z});
        Vec3<double> wi_std = normalize(Vec3<double>{wi.x * a, wi.y * b, wi.z});
        double d = dot(h_std, wi_std);
        Vec3<double> c{2.0 * d * h_std.x - wi_std.x, 2.0 * d * h_std.y - wi_std.y,
                       2.0 * d * h_std.z - wi_std.z};
        u2[i] = 1.0 - (c.z + wi_std.z) / (1.0 + wi_std.z);
        double t = std::atan2(c.y, c.x) / (2.0 * kPi);
        u1[i] = t < 0.0 ? t + 1.0 : t;
    });
    return 0;
}

// Rough-dielectric sampler over tuples (wi, alpha) with one relative index
// eta: outputs wo, the pdf at wo, the weight f |wo.n| / pdf, the lobe (0
// reflection, 1 transmission) and the visible normal h.  Uniforms are given
// (u1, u2, u3 all non-NULL) or drawn from the dielectric stream.  Inputs
// outside the domain (wi_z <= 0, alpha <= 0) give wo = (0, 0, 1), h = (0, 0, 1),
// pdf = weight = 0, lobe = -1.
int32_t orc_dielectric_sample(int64_t n, const double* wix, const double* wiy, const double* wiz,
                              const double* ax, const double* ay, double eta, const double* u1,
                              const double* u2, const double* u3, uint64_t seed,
                              uint64_t index_base, double* wox, double* woy, double* woz,
                              double* pdf, double* weight, int32_t* lobe, double* hx, double* hy,
                              double* hz, int32_t nthreads) {
    if (n < 0 || !(eta > 0.0) || eta == 1.0) return -1;
    if ((u1 == nullptr) != (u2 == nullptr) || (u1 == nullptr) != (u3 == nullptr)) return -1;
    parallel_for(n, nthreads, [&](int64_t i) {
        Vec3<double> wi{wix[i], wiy[i], wiz[i]};
        double a = ax[i], b = ay[i];
        double r1, r2, r3;
        if (u1 != nullptr) {
            r1 = u1[i]; r2 = u2[i]; r3 = u3[i];
        } else {
            dielectric_uniforms(seed, 0u, index_base + (uint64_t)i, &r1, &r2, &r3);
        }
        if (!(wi.z > 0.0) || !(a > 0.0) || !(b > 0.0)) {
            wox[i] = 0.0; woy[i] = 0.0; woz[i] = 1.0;
            pdf[i] = 0.0; weight[i] = 0.0; lobe[i] = -1;
            if (hx) { hx[i] = 0.0; hy[i] = 0.0; hz[i] = 1.0; }
            return;
        }
        DielectricSample s = dielectric_sample(r1, r2, r3, wi, a, b, eta);
        wox[i] = s.wo.x; woy[i] = s.wo.y; woz[i] = s.wo.z;
        pdf[i] = s.pdf; weight[i] = s.weight; lobe[i] = s.lobe;
        if (hx) { hx[i] = s.h.x; hy[i] = s.h.y; hz[i] = s.h.z; }
    });
    return 0;
}

// Dielectric pdf and BSDF at caller-given (wi, wo, alpha), one eta; either
// output may be NULL.
int32_t orc_dielectric_eval(int64_t n, const double* wix, const double* wiy, const double* wiz,
                            const double* wox, const double* woy, const double* woz,
                            const double* ax, const double* ay, double eta, double* pdf,
                            double* bsdf, int32_t nthreads) {
    if (n < 0 || !(eta > 0.0) || eta == 1.0) return -1;
    parallel_for(n, nthreads, [&](int64_t i) {
        Vec3<double> wi{wix[i], wiy[i], wiz[i]}, wo{wox[i], woy[i], woz[i]};
        if (pdf) pdf[i] = dielectric_pdf(wi, wo, ax[i], ay[i], eta);
        if (bsdf) bsdf[i] = (ax[i] > 0.0 && ay[i] > 0.0) ? dielectric_bsdf(wi, wo, ax[i], ay[i], eta) : 0.0;
    });
    return 0;
}

// Unpolarised Fresnel reflectance, element-wise.
void orc_fresnel_dielectric(int64_t n, const double* cos_i, double eta, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = fresnel_dielectric(cos_i[i], eta);
}

// Raw uniforms of the dielectric stream (tuple indices index_base + i).
void orc_dielectric_uniforms(int64_t n, uint64_t seed, uint64_t index_base, double* u1,
                             double* u2, double* u3) {
    for (int64_t i = 0; i < n; ++i)
        dielectric_uniforms(seed, 0u, index_base + (uint64_t)i, u1 + i, u2 + i, u3 + i);
}

int32_t orc_hardware_threads(void) {
    return (int32_t)std::max(1u, std::thread::hardware_concurrency());
}

}  // extern "C"
