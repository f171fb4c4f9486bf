/*
 * capvndf -- spherical-cap sampling of visible GGX normals on MI355X (gfx950).
 *
 * C ABI of libcapvndf.so.  Method: J. Dupuy and A. Benyoub, "Sampling Visible
 * GGX Normals with Spherical Caps" (arXiv 2306.05044).  Section, equation and
 * appendix references below are to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are caller-owned DEVICE pointers (for example a torch tensor's
 *    data_ptr()), FP32 unless stated, contiguous, at least 4-byte aligned.
 *    Structure-of-arrays layout: one array per vector component.
 *    16-byte alignment of every array (and, for vndf_sample, an even
 *    index_base) selects the vectorised path; otherwise a scalar path gives
 *    identical results.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls only enqueue work: they return before the GPU has finished and
 *    never synchronise.  Enqueued work reads inputs and writes outputs
 *    asynchronously, so buffers must stay alive until the stream reaches it.
 *  - Element-wise calls take any n >= 0 that fits in memory: a call longer
 *    than 2^31 elements is enqueued as consecutive launches of 2^31 elements
 *    (results identical to one launch; a HIP error in a later launch leaves
 *    the earlier ones enqueued).  The table estimators take per-cell
 *    sample counts (see albedo_workspace_size) and fewer than 2^24 cells
 *    per call.
 *  - The library never allocates on these calls, except the batch-plan calls
 *    (which own their chunk tables, partial buffers and graph).
 *  - Return value: CAPVNDF_OK (0) or a negative CAPVNDF_ERR_* code.  All
 *    argument checks happen on the host before any launch; on error nothing
 *    is enqueued and capvndf_last_error() describes the problem (the message
 *    is per thread and kept until the next failing call on that thread).
 *    No C++ exception crosses the ABI.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *    (lo32(seed), hi32(seed)) and counter (lo32(k>>1), unit, tag, hi32(k>>1));
 *    sample k takes words (w0, w1) when k is even and (w2, w3) when odd, and
 *    u = (w >> 8) * 2^-24.  Tags: 2 = vndf_sample (unit 0, k = index_base + i),
 *    3 = albedo estimators (unit = cell or job index, k = sample index).
 *    dielectric_sample needs three uniforms per tuple and takes a whole block
 *    per tuple instead: counter (lo32(k), 0, 5, hi32(k)), words 0, 1, 2.
 *  - Domain: directions need w_z > 0 and roughness alpha > 0.  Elements
 *    outside it give h = (0, 0, 1) and pdf = 0; albedo cells or jobs outside
 *    it give 0 values and 0 gradients.  Inputs in the documented ranges never
 *    produce NaN.
 */
#ifndef CAPVNDF_H
#define CAPVNDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CAPVNDF_OK 0
#define CAPVNDF_ERR_NULL_PTR (-1)
#define CAPVNDF_ERR_BAD_SIZE (-2)
#define CAPVNDF_ERR_MISALIGNED (-3)
#define CAPVNDF_ERR_BAD_METHOD (-4)
#define CAPVNDF_ERR_WORKSPACE (-5)
#define CAPVNDF_ERR_HIP (-6)
#define CAPVNDF_ERR_BAD_ARG (-7)

/* Hemisphere routine used inside the general VNDF sampler (Sec. 2, steps 1-3). */
#define CAPVNDF_CAP 0      /* spherical cap, Sec. 3.3 (the paper's method)   */
#define CAPVNDF_DISK2018 1 /* Heitz 2018 cross section, Sec. 2 (baseline)    */
#define CAPVNDF_CAP_F64 2  /* spherical cap evaluated in double precision   */

/* Version of this ABI (major * 10000 + minor * 100 + patch): 3.2.0.  Minor 2
 * of major 3 added albedo_value_and_grad_noalloc; minor 1 added a 32-byte
 * horizon record per slot to the workspace of the gradient entry points
 * (albedo_workspace_size covers it); major 3
 * gave the table estimators per-cell device sample counts and
 * albedo_workspace_size its (ncells, host counts, with_grad) form; major 2
 * added the `dynamic` field to capvndf_tiling (a layout change) and the
 * CAPVNDF_CAP_F64 method; minor 1 of major 2 added albedo_view_from_angles
 * and albedo_apply_jacobian. */
#define CAPVNDF_VERSION 30200
int32_t capvndf_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* capvndf_last_error(void);

/*
 * vndf_sample -- draw n GGX visible normals, Sec. 2 "Importance Sampling"
 * (warp wi by M^-1 = diag(ax, ay, 1), sample the hemisphere's visible normals,
 * warp back by M^-T and normalise) with the hemisphere routine `method`:
 * CAPVNDF_CAP = Sec. 3.3 (uniform point c on the cap z in (-z_i, 1], half
 * vector c + wi), CAPVNDF_DISK2018 = Heitz's cross-section sampler,
 * CAPVNDF_CAP_F64 = the cap sampler evaluated in double precision from the
 * same FP32 inputs and uniforms (same samples; FP32 arithmetic loses about
 * 2^-24 (1 + max(ax, ay)/L + 1/|c + wi|) relatively, L = |M^-T (c + wi)|,
 * which exceeds 2e-6 near grazing half vectors; in double every output is
 * within 2e-6, in practice a few ulps, of the exact sample; 1.00-1.05x the
 * FP32 method's time on this part).
 *
 *   n            number of tuples (>= 0; 0 enqueues nothing)
 *   wix,wiy,wiz  view directions wi (need not be unit; w_z > 0)       [n]
 *   ax, ay       roughness alpha_x, alpha_y (> 0); may alias          [n]
 *   u1, u2       uniforms in [0, 1) (u1 -> azimuth, u2 -> height, u2 = 0 at
 *                the cap's apex; values outside [0, 1) give unspecified
 *                results), or both NULL to draw them from Philox tag 2 at
 *                sample index index_base + i                            [n]
 *   seed         Philox key (ignored when u1/u2 are given)
 *   index_base   offset of this call in the Philox stream
 *   hx, hy, hz   out: unit microfacet normals h                        [n]
 *   pdf          out (nullable): VNDF pdf of Eq. (1) at the sample,
 *                G1(wi) max(0, wi.h) D(h) / w_z, per unit solid angle  [n]
 * Errors: NULL_PTR (a required array is NULL or only one of u1/u2 given),
 * BAD_SIZE (n < 0), MISALIGNED (not 4-byte aligned), BAD_METHOD, HIP.
 */
int32_t vndf_sample(int64_t n, const float* wix, const float* wiy, const float* wiz,
                    const float* ax, const float* ay, const float* u1, const float* u2,
                    uint64_t seed, uint64_t index_base, int32_t method, float* hx, float* hy,
                    float* hz, float* pdf, void* stream);

/*
 * vndf_pdf -- VNDF pdf of Eq. (1) (a linearly transformed hemisphere VNDF,
 * Eqs. (2)-(4)) at caller-given unit normals h seen from wi:
 * pdf = G1(wi) max(0, wi.h) D(h) / w_z with D and G1 of Appendix A.
 *
 *   n; wix,wiy,wiz [n]; hx,hy,hz unit normals [n]; ax, ay [n]; pdf out [n].
 * pdf is 0 when w_z <= 0, h_z <= 0, wi.h <= 0 or alpha <= 0.  Evaluated in
 * double precision with an exact wi.h, so grazing normals keep full relative
 * accuracy (the result is the FP32 rounding of the exact value up to a few
 * ulps).
 * Errors: NULL_PTR, BAD_SIZE, MISALIGNED, HIP.
 */
int32_t vndf_pdf(int64_t n, const float* wix, const float* wiy, const float* wiz,
                 const float* hx, const float* hy, const float* hz, const float* ax,
                 const float* ay, float* pdf, void* stream);

/*
 * vndf_inverse -- inverse of the cap sampler (vndf_sample with CAPVNDF_CAP):
 * the uniforms (u1, u2) that produce a given visible normal h seen from wi.
 * By the reflection law and the half-vector relation of Sec. 3.2 the
 * hemisphere normal n = M^T h / |M^T h| reflects wi_std into the cap point
 * c = 2 (n . wi_std) n - wi_std, whose height and azimuth invert the cap
 * parameterisation of Sec. 3.3.  Useful to map normals back to primary
 * sample space (e.g. to reuse or mutate paths).
 *
 *   n; wix,wiy,wiz [n]; hx,hy,hz unit visible normals [n]; ax, ay [n];
 *   u1, u2 [n] out: in [0, 1) (u2 clamped there, since rounding can
 *   carry a normal at the rim of the cap past 1); both -1 outside the
 *   domain (w_z <= 0, alpha <= 0, h_z <= 0 or wi.h <= 0).  u1 is undefined
 *   at the apex of the cap (u2 = 0) and returned as atan2 gives it there.
 * The geometry is evaluated in double and the azimuth in FP32: u2 is the
 * rounding of the exact value, u1 within a few 2^-24 turns of it.
 * Errors: NULL_PTR, BAD_SIZE, MISALIGNED, HIP.
 */
int32_t vndf_inverse(int64_t n, const float* wix, const float* wiy, const float* wiz,
                     const float* hx, const float* hy, const float* hz, const float* ax,
                     const float* ay, float* u1, float* u2, void* stream);

/*
 * dielectric_sample -- sampling of a rough dielectric interface (reflection
 * and transmission) with the same spherical-cap VNDF sampler.  The paper
 * benchmarks its sampler on rough dielectrics and takes their model from
 * Walter et al. 2007: a visible normal h is drawn from the VNDF seen from wi
 * (Sec. 3.3), the lobe is reflection with probability F (unpolarised Fresnel
 * reflectance at wi . h, 1 under total internal reflection), and wi is then
 * reflected (wo = 2 (wi.h) h - wi) or refracted by Snell's law about h.
 *
 *   n            number of tuples (>= 0)
 *   wix,wiy,wiz  unit incident directions on the upper side, w_z > 0      [n]
 *   ax, ay       roughness                                               [n]
 *   u1, u2, u3   caller-given uniforms in [0, 1) (u1 azimuth, u2 height on
 *                the cap, u3 the lobe), or all three NULL to draw them from
 *                the Philox block with counter (lo32(k), 0, 5, hi32(k)),
 *                k = index_base + i, words 0, 1, 2                       [n]
 *   eta          relative index of refraction n_lower / n_upper: finite,
 *                > 0 and != 1 (1.5 for glass seen from air, 1/1.5 for air
 *                seen from inside glass with the frame flipped)
 *   seed, index_base  Philox key and stream offset (ignored with explicit u)
 *   wox,woy,woz  out: unit outgoing directions                           [n]
 *   pdf          out: density of wo per unit solid angle, the lobe
 *                probability times the VNDF times |dh/dwo|               [n]
 *   weight       out: f |wo_z| / pdf = G2(wi, wo) / G1(wi), with the BTDF of
 *                Walter et al. (its eta^2 factor included, i.e. no
 *                radiance rescaling by 1/eta^2)                          [n]
 * A reflected direction below the surface or a transmitted one above it is
 * no sample: its pdf and weight are 0 (wo is still written).  Inputs outside
 * the domain (w_z <= 0, alpha <= 0) give wo = (0, 0, 1), pdf = weight = 0.
 * Errors: NULL_PTR (a required array is NULL or only some of u1, u2, u3
 * given), BAD_SIZE (n < 0), MISALIGNED, BAD_ARG (eta), HIP.
 */
int32_t dielectric_sample(int64_t n, const float* wix, const float* wiy, const float* wiz,
                          const float* ax, const float* ay, const float* u1, const float* u2,
                          const float* u3, float eta, uint64_t seed, uint64_t index_base,
                          float* wox, float* woy, float* woz, float* pdf, float* weight,
                          void* stream);

/*
 * dielectric_pdf -- the density of dielectric_sample at caller-given unit
 * pairs (wi, wo), for multiple importance sampling: with the half vector
 * h = wi + wo (wo above) or h = -(wi + eta wo) (wo below, Walter et al.'s
 * generalised half vector), normalised to the upper side,
 *   pdf = F(wi.h) VNDF(h) / (4 |wo.h|)                         (reflection),
 *   pdf = (1 - F(wi.h)) VNDF(h) eta^2 |wo.h| / (wi.h + eta wo.h)^2 (transmission).
 * 0 when wi.h <= 0, when a reflected wo lies behind h (wo.h <= 0) or a
 * transmitted one in front of it (wo.h >= 0), for wo_z = 0 and outside the
 * domain.  Evaluated in double precision at the given vectors as written
 * (FP32 directions are unit only up to rounding): the result is the FP32
 * rounding of that value up to a few ulps.
 *   n; wix,wiy,wiz [n]; wox,woy,woz [n]; ax, ay [n]; eta as above; pdf out [n].
 * Errors: NULL_PTR, BAD_SIZE, MISALIGNED, BAD_ARG (eta), HIP.
 */
int32_t dielectric_pdf(int64_t n, const float* wix, const float* wiy, const float* wiz,
                       const float* wox, const float* woy, const float* woz, const float* ax,
                       const float* ay, float eta, float* pdf, void* stream);

/*
 * Sample counts of the table estimators.  Appendix A's estimator of a cell
 * (one outgoing direction) averages N samples; every cell has its own N,
 * given as a DEVICE array `nsamples` of int64 (8-byte aligned), N in
 * [0, 2^40).  A cell of N samples is cut into ceil(ceil(N / 2) / 8192)
 * chunks of 16384 samples.  A call gives each cell a number of slots (blocks)
 * chosen on the host from the cell count and the workspace: slot s of a cell
 * sums the cell's chunks s, s + slots, ... into one compensated partial, and
 * the partials are merged in slot order, so results are bitwise reproducible
 * for the same inputs and workspace size.  A count outside [0, 2^40) gives
 * NaN outputs for that cell; a count of 0 gives 0.  At most 2^24 - 1 cells
 * per call.
 *
 * albedo_workspace_size -- bytes of device workspace for ncells cells:
 *   nsamples_host [ncells] HOST copy of the per-cell counts, or NULL.  With
 *                 the counts, the size covers slots up to the largest cell's
 *                 chunk count only (fewer, fuller blocks); without, the
 *                 most slots a call of ncells cells uses.
 *   with_grad     0: enough for albedo_estimate, albedo_value_and_grad
 *                 without gradients and radiance_estimate; 1: enough for
 *                 every table estimator (two or four partial sums per slot,
 *                 and with gradients a 32-byte horizon record per slot).
 * Any workspace of at least ncells * (8 * partial sums of the call, + 32 with
 * gradients) bytes works; a larger one (up to this size) lets the call use
 * more slots.
 * Returns 0 for ncells <= 0, ncells >= 2^24, with_grad not 0 or 1, or a host
 * count outside [0, 2^40).
 */
size_t albedo_workspace_size(int64_t ncells, const int64_t* nsamples_host, int32_t with_grad);

/*
 * albedo_estimate -- directional albedo per cell: the Monte Carlo estimator
 * of Appendix A ("Importance Sampling Using the GGX VNDF") with L == 1.  Each
 * sample draws h with the cap sampler from the view direction wo, reflects wo
 * about h (reflection law of Sec. 3.2) and weighs the result by
 * f_r |cos theta_l| / PDF = F(wo.h) G2(wo, wl) / G1(wo); reflections at or
 * below the horizon weigh 0 but count.  With Schlick's Fresnel
 * F = F0 + (1 - F0)(1 - wo.h)^5 the albedo is linear in F0, so one stream
 * gives both sums:
 *   s_f1[c] = (1/N_c) sum G2/G1,  s_f5[c] = (1/N_c) sum G2/G1 (1 - wo.h)^5,
 *   A(F0)   = F0 s_f1 + (1 - F0) s_f5.
 * Sums are compensated (TwoSum) and reduced in a fixed order.
 *
 *   ncells               number of cells (>= 0)
 *   wox,woy,woz [ncells] view directions (normalised internally; wo_z > 0)
 *   ax, ay      [ncells] roughness
 *   nsamples    [ncells] device int64: samples N_c of each cell (see above)
 *   seed                 Philox key; cell c uses unit c of tag 3
 *   s_f1, s_f5  [ncells] out
 *   workspace            device scratch, 16-byte aligned, of
 *                        albedo_workspace_size(ncells, counts, 0) bytes (at
 *                        least ncells * 16)
 * Errors: NULL_PTR, BAD_SIZE, MISALIGNED, WORKSPACE (too small), HIP.
 */
int32_t albedo_estimate(int64_t ncells, const float* wox, const float* woy, const float* woz,
                        const float* ax, const float* ay, const int64_t* nsamples, uint64_t seed,
                        float* s_f1, float* s_f5, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * albedo_estimate_backward -- pathwise (reparameterised) adjoint of the
 * estimator above for A(F0) = (1/N) sum F G2/G1: the same samples, recomputed
 * from the Philox counter (nothing is stored), differentiated at fixed
 * (u1, u2) through the stretch, the cap map, the unstretch, the reflection,
 * G1/G2 and Fresnel.  The weight is continuous where the reflection crosses
 * the horizon, so the pathwise gradient is unbiased.
 *
 *   (same cell inputs, nsamples and seed as albedo_estimate)
 *   f0          [ncells] Fresnel F0 per cell (NULL = 1)
 *   grad_albedo [ncells] upstream gradient dL/dA (NULL = 1)
 *   grad_ax, grad_ay [ncells] out: dL/dA * dA/d alpha_x, dA/d alpha_y
 *   grad_theta_o     [ncells] out: dL/dA * dA/d theta_o, the derivative along
 *                    the meridian of wo at fixed azimuth
 *                    (dwo/dtheta = (cos t cos p, cos t sin p, -sin t); at the
 *                    pole the azimuth is taken as 0)
 *   workspace        albedo_workspace_size(ncells, counts, 1) bytes (at
 *                    least ncells * 56)
 * The samples whose FP32 reflection lies within rounding of the horizon,
 * where the weight's slope jumps, or whose conditioning is too poor for FP32
 * (a few in 10^5) are evaluated again in double precision by a second kernel
 * on the same stream, which replaces their FP32 terms.
 * Errors: as albedo_estimate.
 */
int32_t albedo_estimate_backward(int64_t ncells, const float* wox, const float* woy,
                                 const float* woz, const float* ax, const float* ay,
                                 const int64_t* nsamples, uint64_t seed, const float* f0,
                                 const float* grad_albedo, float* grad_ax, float* grad_ay,
                                 float* grad_theta_o, void* workspace, size_t workspace_bytes,
                                 void* stream);

/*
 * albedo_value_and_grad -- A(F0) per cell for the cell's own F0 (the same
 * estimator and Philox streams as albedo_estimate) and, when the three
 * gradient outputs are given, dA/d alpha_x, dA/d alpha_y and dA/d theta_o
 * (definitions as in albedo_estimate_backward) from the same pass over the
 * samples.  Each cell's value depends only on its own parameters, so these
 * three arrays are the whole Jacobian: a caller that needs the gradient of a
 * loss multiplies them by dL/dA instead of running the backward pass.
 *
 *   (cell inputs, nsamples, seed as albedo_estimate)
 *   f0          [ncells] Fresnel F0 per cell (NULL = 1)
 *   albedo      [ncells] out: A(F0)
 *   grad_ax, grad_ay, grad_theta_o [ncells] out, all NULL for values only
 *   workspace   albedo_workspace_size(ncells, counts, 1) bytes (at least
 *               ncells * 64 with gradients, ncells * 8 without)
 * With gradients, near-horizon samples are evaluated again in double
 * precision as in albedo_estimate_backward.
 * Errors: as albedo_estimate; NULL_PTR if only some gradient outputs are given.
 */
int32_t albedo_value_and_grad(int64_t ncells, const float* wox, const float* woy,
                              const float* woz, const float* ax, const float* ay,
                              const int64_t* nsamples, uint64_t seed, const float* f0,
                              float* albedo, float* grad_ax, float* grad_ay, float* grad_theta_o,
                              void* workspace, size_t workspace_bytes, void* stream);

/*
 * albedo_value_and_grad_noalloc -- albedo_value_and_grad without a workspace
 * argument, for callers that cannot allocate device memory: code that must
 * not call hipMalloc while it enqueues work (a stream being captured into a
 * graph, a tight serving loop, a harness that forbids allocation).  It
 * allocates nothing: its partial sums and horizon records live in a 16 MiB
 * device buffer of the library (a file-scope array, one copy per device,
 * held until the process ends), whose address is looked up once per device
 * on the first call there.  Same arguments, results and errors as
 * albedo_value_and_grad (the same kernels, so the same bits as a call with a
 * workspace of the size this buffer gives), except:
 *   - at most 262144 cells per call with gradients (64 bytes per cell at one
 *     slot) and 2097152 without (8 bytes); more gives BAD_SIZE;
 *   - the slot count is the one a 16 MiB workspace allows;
 *   - every call on one device shares the buffer: calls that overlap on one
 *     device (two streams, two host threads) race on it and must be ordered
 *     by the caller.  Nothing needs clearing between calls: each call writes
 *     every partial and record it reads.
 */
int32_t albedo_value_and_grad_noalloc(int64_t ncells, const float* wox, const float* woy,
                                      const float* woz, const float* ax, const float* ay,
                                      const int64_t* nsamples, uint64_t seed, const float* f0,
                                      float* albedo, float* grad_ax, float* grad_ay,
                                      float* grad_theta_o, void* stream);

/*
 * radiance_estimate -- direct illumination per cell: the Monte Carlo
 * estimator of Appendix A ("Importance Sampling Using the GGX VNDF") with an
 * incident radiance L(w_b) that is a sum of spherical-Gaussian lobes,
 *   L(w) = sum_k lambda_k exp(kappa_k (mu_k . w - 1)),
 * i.e. (1/N) sum F(wo.h) G2/G1 L(wl) over the same samples (Philox tag 3,
 * unit = cell index) as albedo_estimate.  A constant radiance (kappa = 0)
 * gives lambda times the albedo.
 *
 *   (cell inputs, nsamples, seed as albedo_estimate)
 *   f0          [ncells] Fresnel F0 per cell (NULL = 1)
 *   lobes       device FP32 [5 * nlobes]: (mu_x, mu_y, mu_z, kappa, lambda)
 *               per lobe, mu unit, kappa >= 0 (the lobe's FP32 relative
 *               error grows as kappa * 2^-24)
 *   nlobes      0 .. 8 (0 gives zero radiance)
 *   radiance    [ncells] out
 *   workspace   albedo_workspace_size(ncells, counts, 0) bytes (at least
 *               ncells * 8)
 * Errors: as albedo_estimate; BAD_SIZE for nlobes outside [0, 8].
 */
int32_t radiance_estimate(int64_t ncells, const float* wox, const float* woy, const float* woz,
                          const float* ax, const float* ay, const float* f0,
                          const int64_t* nsamples, uint64_t seed, const float* lobes,
                          int32_t nlobes, float* radiance, void* workspace,
                          size_t workspace_bytes, void* stream);

/*
 * albedo_view_from_angles -- view directions from spherical angles,
 *   wo = (sin theta cos phi, sin theta sin phi, cos theta),
 * the parametrisation whose polar derivative albedo_estimate_backward and
 * albedo_value_and_grad report (theta_o is the angle to the macro-normal,
 * Sec. 2's frame with the surface normal along +z).  FP32 with the library's
 * sincosf (a few ulps).
 *
 *   n                    number of directions (>= 0)
 *   theta_o, phi_o [n]   angles in radians (device, FP32)
 *   wox, woy, woz  [n]   out (device, FP32); may not alias the inputs
 * Errors: BAD_SIZE (n < 0), NULL_PTR, MISALIGNED, HIP.
 */
int32_t albedo_view_from_angles(int64_t n, const float* theta_o, const float* phi_o, float* wox,
                                float* woy, float* woz, void* stream);

/*
 * albedo_apply_jacobian -- the chain rule through the per-cell Jacobian of
 * the albedo (each cell's A depends only on that cell's parameters, so the
 * Jacobian is diagonal): with g = dL/dA,
 *   grad_ax = g * d_ax,  grad_ay = g * d_ay,  grad_theta_o = g * d_theta_o
 * for the derivatives from albedo_value_and_grad, and
 *   grad_f0 = g * (s_f1 - s_f5),
 * dA/dF0 exactly, from the two sums of albedo_estimate on the same stream
 * (Schlick's F is linear in F0).  One correctly rounded FP32 multiply per
 * output (and one subtraction for F0).
 *
 *   n                     number of cells (>= 0)
 *   grad_albedo [n]       g (device, FP32)
 *   d_ax, d_ay, d_theta_o [n] each NULL to skip that output
 *   s_f1, s_f5  [n]       both NULL to skip grad_f0
 *   grad_ax, grad_ay, grad_theta_o, grad_f0 [n] out; NULL exactly where
 *                         the matching input is NULL; distinct from each
 *                         other, but each may alias any input (every input
 *                         of an element is read before its outputs are
 *                         written)
 * Errors: BAD_SIZE (n < 0), NULL_PTR (also for an output without its input
 * or the reverse), MISALIGNED, HIP.
 */
int32_t albedo_apply_jacobian(int64_t n, const float* grad_albedo, const float* d_ax,
                              const float* d_ay, const float* d_theta_o, const float* s_f1,
                              const float* s_f5, float* grad_ax, float* grad_ay,
                              float* grad_theta_o, float* grad_f0, void* stream);

/*
 * Batched estimation of many jobs with uneven sample counts (forward value
 * A_j(F0_j) plus, with with_grad, dA_j/d alpha_x, dA_j/d alpha_y and
 * dA_j/d theta_o), in one persistent launch plus a fixed-order finishing pass
 * (and, with gradients, the horizon fix pass of albedo_estimate_backward
 * between them), captured once into a HIP graph and replayed by
 * albedo_batch_run.  Job j uses unit j of tag 3, so its values equal
 * albedo_estimate/backward on that job.
 *
 * Tiling: block size, pairs of samples per thread per chunk (multiple of 8),
 * resident blocks per compute unit, who owns a chunk -- the whole block
 * (per_wave = 0; block-wide reduction through LDS) or a single wavefront
 * (per_wave = 1; smaller chunks, wave-only reduction, so short jobs occupy 64
 * lanes instead of a block) -- and how chunks reach their owners: a static
 * partition balanced by sample count (dynamic = 0) or the next index from a
 * device counter (dynamic = 1; balances run-time differences, still
 * deterministic since every chunk has its own result slot).
 */
typedef struct capvndf_tiling {
    int32_t block;            /* 256 or 512 threads                          */
    int32_t pairs_per_thread; /* chunk = owner lanes * pairs_per_thread pairs */
    int32_t blocks_per_cu;    /* persistent grid = CUs * blocks_per_cu        */
    int32_t per_wave;         /* 0: a block owns a chunk; 1: a wavefront does */
    int32_t dynamic;          /* 0: static chunk ranges; 1: chunk counter      */
} capvndf_tiling;

typedef struct capvndf_batch_plan capvndf_batch_plan;

/*
 * albedo_batch_plan_create -- plan the batch and capture its graph.
 *   njobs                 number of jobs (>= 1)
 *   wox..ay      [njobs]  device job parameters (as albedo_estimate)
 *   f0           [njobs]  device Fresnel F0 per job (NULL = 1)
 *   nsamples_host[njobs]  HOST array of sample counts (>= 0, < 2^40)
 *   seed                  Philox key
 *   with_grad             0: values only; 1: values and gradients
 *   albedo       [njobs]  device out: A_j(F0_j)
 *   grad_ax, grad_ay, grad_theta_o [njobs] device out (ignored if !with_grad)
 *   tiling                NULL: the tuned tiling cached for this problem
 *                         signature (CAPVNDF_TUNE_CACHE file) or the default
 *                         {256, 32, 8, 0, 0}
 *   stream                unused: the graph is captured on a private stream
 *                         of the current device, which the plan belongs to
 *   out                   receives the plan
 * The plan keeps the pointers: they must stay valid while the plan is used,
 * and new buffers need a new plan.  Errors: NULL_PTR, BAD_SIZE, BAD_ARG, HIP.
 */
int32_t albedo_batch_plan_create(int64_t njobs, const float* wox, const float* woy,
                                 const float* woz, const float* ax, const float* ay,
                                 const float* f0, const int64_t* nsamples_host, uint64_t seed,
                                 int32_t with_grad, float* albedo, float* grad_ax, float* grad_ay,
                                 float* grad_theta_o, const capvndf_tiling* tiling, void* stream,
                                 capvndf_batch_plan** out);

/* Replay the plan's graph on `stream` (one hipGraphLaunch).  The current
 * device must be the plan's.  A plan's partials (and, with dynamic = 1, its
 * chunk counter, which the graph resets with a kernel before each launch)
 * belong to the plan: replays of one plan must not overlap (issue them on one
 * stream or order them with events); different plans may run concurrently.
 * Errors: NULL_PTR, BAD_ARG (other device), HIP. */
int32_t albedo_batch_run(capvndf_batch_plan* plan, void* stream);

/* Same jobs and outputs as albedo_batch_run, launched the per-request way:
 * per job one albedo_value_and_grad-style estimate kernel (with gradients
 * followed by its horizon fix kernel) plus its finishing kernel, no graph.  The baseline the batch is measured against.  Errors as
 * albedo_batch_run, and BAD_SIZE (nothing enqueued) when a job has 2^24 or
 * more chunks of 16384 samples, more than one launch of this path covers. */
int32_t albedo_batch_run_per_request(capvndf_batch_plan* plan, void* stream);

/* Tiling and chunk statistics of a plan. */
int32_t albedo_batch_plan_info(const capvndf_batch_plan* plan, capvndf_tiling* tiling,
                               int64_t* nchunks, int64_t* total_samples);

/* Free the plan, its device buffers and its graph (NULL is a no-op).  It
 * first waits for the plan's last albedo_batch_run or
 * albedo_batch_run_per_request to finish (an event recorded by each). */
void albedo_batch_plan_destroy(capvndf_batch_plan* plan);

/*
 * albedo_batch_autotune -- time candidate tilings on the given jobs (replays
 * on `stream`, synchronising it) and return the fastest in *best and its mean
 * time per run in *best_ms.  When CAPVNDF_TUNE_CACHE names a file, the result
 * is stored there under the problem signature for later plans.  Candidates:
 * block 256 or 512 threads x pairs_per_thread 8..64 (block-owned chunks) or
 * 8..128 (wavefront-owned chunks) x blocks_per_cu 2..16 (2..8 for 512), each
 * with static and dynamic chunk assignment.  Candidates the planner refuses
 * for their size (more than 2^31 - 2 chunks) are skipped; BAD_SIZE if all are.
 * Arguments as albedo_batch_plan_create; outputs are overwritten.
 */
int32_t albedo_batch_autotune(int64_t njobs, const float* wox, const float* woy,
                              const float* woz, const float* ax, const float* ay,
                              const float* f0, const int64_t* nsamples_host, uint64_t seed,
                              int32_t with_grad, float* albedo, float* grad_ax, float* grad_ay,
                              float* grad_theta_o, void* stream, capvndf_tiling* best,
                              float* best_ms);

/*
 * Random-number and measurement hooks.
 *
 * capvndf_uniforms -- the (u1, u2) of samples k0 .. k0+n-1 of stream
 * (seed, tag, unit), written to device arrays u1, u2 [n] (FP32, exact).
 */
int32_t capvndf_uniforms(uint64_t seed, uint32_t tag, uint32_t unit, uint64_t k0, int64_t n,
                         float* u1, float* u2, void* stream);

/* capvndf_philox_blocks -- raw Philox4x32-10 of n counters: ctr and out are
 * device uint32 arrays of 4n words (counter i at 4i..4i+3); key is (k0, k1). */
int32_t capvndf_philox_blocks(int64_t n, const uint32_t* ctr, uint32_t key0, uint32_t key1,
                              uint32_t* out, void* stream);

/*
 * vndf_microbench -- register-resident sampler benchmark in the shape of the
 * paper's GPU benchmark (Sec. 4, "GPU Synthetic Benchmark": the general
 * sampler called 64 times per lane): each of `lanes` lanes draws its view
 * direction and roughness once, then calls the sampler `iters` times on
 * cheap low-discrepancy uniforms and a view elevation that changes every call,
 * folding h into one word written to out[lane] (device, [lanes]).  method:
 * CAPVNDF_CAP, CAPVNDF_DISK2018 or CAPVNDF_CAP_F64; lanes <= 2^31.
 */
int32_t vndf_microbench(int32_t method, int64_t lanes, int32_t iters, uint64_t seed,
                        uint32_t* out, void* stream);

/*
 * estimator_microbench -- register-resident benchmark of the estimators'
 * per-sample arithmetic: each of `lanes` lanes draws one cell (view uniform
 * over the hemisphere, alpha_x, alpha_y = 10^(-2U)) and runs the per-sample
 * code of one table estimator on `pairs` Philox pairs of its own stream
 * (tag 3, unit = lane index) into plain per-lane sums, written as one word
 * to out[lane] (device, [lanes]).  No loads in the loop, no compensated sums
 * and no cross-lane reductions: the issue rate of that instruction mix with
 * nothing else in the way, against which the table kernels are measured.
 * kind 0: albedo_estimate's two sums; 1: albedo_value_and_grad's value and
 * adjoint; 2: radiance_estimate's term under the 4 lobes in `lobes` (device
 * FP32 [20], as radiance_estimate's; ignored for other kinds).
 * Errors: BAD_SIZE (lanes outside [0, 2^31], pairs < 0), BAD_ARG (kind),
 * NULL_PTR, MISALIGNED, HIP.
 */
int32_t estimator_microbench(int32_t kind, int64_t lanes, int32_t pairs, uint64_t seed,
                             const float* lobes, uint32_t* out, void* stream);

/*
 * capvndf_stream_probe -- plain streaming kernels with the sampler's arrays,
 * vector width and launch shape, to measure the achievable HBM bandwidth and
 * calibrate hardware byte counters.  mode 0: the sampler's traffic (5 FP32
 * arrays read, 4 written: out0 = in0 + in4, out1..3 = in1..3); mode 1: the
 * five reads only (outputs untouched for finite inputs); mode 2: the four
 * writes only (index-derived values; inputs unread).  All nine arrays must be
 * valid and 16-byte aligned.  Errors: NULL_PTR, BAD_SIZE, MISALIGNED,
 * BAD_ARG (mode), HIP.
 */
int32_t capvndf_stream_probe(int32_t mode, int64_t n, const float* in0, const float* in1,
                             const float* in2, const float* in3, const float* in4, float* out0,
                             float* out1, float* out2, float* out3, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CAPVNDF_H */
