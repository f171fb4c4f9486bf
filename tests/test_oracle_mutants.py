"""The pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's source -- a flipped
sign, swapped operands, a dropped or wrong factor -- builds it, and runs the
oracle pin tests against that build in a subprocess.  The pins pass on the
real oracle (the rest of this suite) and must fail on every mutant.
"""

import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
PINS = ["tests/test_oracle_rng.py", "tests/test_oracle_sampler.py", "tests/test_oracle_pdf.py",
        "tests/test_oracle_albedo.py", "tests/test_oracle_radiance.py",
        "tests/test_oracle_dielectric.py", "tests/test_oracle_horizon_band.py"]

# (name, text in oracle.cpp, replacement)
MUTANTS = [
    ("philox key bump", "k[0] += kPhiloxW0;", "k[0] += kPhiloxW1;"),
    ("philox word order", "uint32_t n1 = lo1;", "uint32_t n1 = hi1;"),
    ("uniform bits", "(double)(w >> 8) * (1.0 / 16777216.0)", "(double)(w >> 9) * (1.0 / 16777216.0)"),
    ("cap height sign", "const T height = T(1.0) - S(u2) * (T(1.0) + wi.z);",
     "const T height = T(1.0) - S(u2) * (T(1.0) - wi.z);"),
    ("u roles swapped", "const T height = T(1.0) - S(u2) * (T(1.0) + wi.z);",
     "const T height = T(1.0) - S(u1) * (T(1.0) + wi.z);"),
    ("cap azimuth from the height's number", "const S azimuth = S(2.0) * pi_of<S>() * S(u1);",
     "const S azimuth = S(2.0) * pi_of<S>() * S(u2);"),
    ("horizon band without the G1 division", "Dual3 w = fresnel_schlick(cd, f0[c]) * g2 / go;",
     "Dual3 w = fresnel_schlick(cd, f0[c]) * g2;"),
    ("no quadruple precision at the cap's rim", "if (cap_conditioning(h, wi, a, b) > kQuadKappa) {",
     "if (cap_conditioning(h, wi, a, b) > 1e300) {"),
    ("half vector drops wi", "return Vec3<T>{wi.x + c.x, wi.y + c.y, wi.z + c.z};",
     "return Vec3<T>{wi.x + c.x, wi.y + c.y, c.z};"),
    ("stretch transposed",
     "Vec3<T> wi_std = normalize(Vec3<T>{wi.x * ax, wi.y * ay, wi.z});\n    Vec3<T> wm_std = method",
     "Vec3<T> wi_std = normalize(Vec3<T>{wi.x * ay, wi.y * ax, wi.z});\n    Vec3<T> wm_std = method"),
    ("unstretch inverted", "return normalize(Vec3<T>{wm_std.x * ax, wm_std.y * ay, wm_std.z});",
     "return normalize(Vec3<T>{wm_std.x / ax, wm_std.y / ay, wm_std.z});"),
    ("pdf Jacobian power", "return vndf_std(wm_std, wi_std) * det / (len * len * len);",
     "return vndf_std(wm_std, wi_std) * det / (len * len * len * len);"),
    ("cross-section area", "T sigma_std(const Vec3<T>& wi) { return (T(1.0) + wi.z) / 2.0; }",
     "T sigma_std(const Vec3<T>& wi) { return (T(1.0) + wi.z); }"),
    ("NDF determinant", "T det = T(1.0) / (ax * ay);\n    T len2", "T det = ax * ay;\n    T len2"),
    ("G2 uncorrelated", "if (!(value(den) > 0.0)) return T(0.0);\n    return gi * go / den;",
     "if (!(value(den) > 0.0)) return T(0.0);\n    return gi * go;"),
    ("Fresnel power", "return f0 + (1.0 - f0) * (m2 * m2 * m);", "return f0 + (1.0 - f0) * (m2 * m2);"),
    ("reflection sign", "Vec3<T> wb{2.0 * c * wm.x - wa.x, 2.0 * c * wm.y - wa.y, 2.0 * c * wm.z - wa.z};",
     "Vec3<T> wb{2.0 * c * wm.x + wa.x, 2.0 * c * wm.y + wa.y, 2.0 * c * wm.z - wa.z};"),
    ("BRDF cosine dropped", "return f * g2 * d / (4.0 * wa.z * wb.z);", "return f * g2 * d / (4.0 * wa.z);"),
    ("estimator pdf G1 dropped", "T pdf = smith_g1(wm, wa, ax, ay) * ggx_ndf(wm, ax, ay) / (4.0 * wa.z);",
     "T pdf = ggx_ndf(wm, ax, ay) / (4.0 * wa.z);"),
    ("dual sqrt derivative", "double f = 0.5 / s;", "double f = 1.0 / s;"),
    ("dual quotient rule", "(a.d[0] - q * b.d[0]) / b.v", "(a.d[0] + q * b.d[0]) / b.v"),
    ("theta tangent sign", "return Vec3<double>{wo.z * wo.x / rho, wo.z * wo.y / rho, -rho};",
     "return Vec3<double>{wo.z * wo.x / rho, wo.z * wo.y / rho, rho};"),
    ("disk warp weight", "const T frac_disk = (T(1.0) + wi.z) / 2.0;",
     "const T frac_disk = (T(1.0) - wi.z) / 2.0;"),
    ("disk basis", "e1 = Vec3<T>{-wi.y * inv, wi.x * inv, T(0.0)};",
     "e1 = Vec3<T>{wi.y * inv, wi.x * inv, T(0.0)};"),
    ("lobe exponent", "l += p[4] * std::exp(p[3] * (c - 1.0));", "l += p[4] * std::exp(p[3] * (1.0 - c));"),
    ("inverse azimuth swapped", "double t = std::atan2(c.y, c.x) / (2.0 * kPi);",
     "double t = std::atan2(c.x, c.y) / (2.0 * kPi);"),
    ("inverse height", "u2[i] = 1.0 - (c.z + wi_std.z) / (1.0 + wi_std.z);",
     "u2[i] = 1.0 - (c.z - wi_std.z) / (1.0 + wi_std.z);"),
    ("radiance at the view", "return radiance(normalize(wb), params, nlobes) * fr * wb.z / pdf;",
     "return radiance(wa, params, nlobes) * fr * wb.z / pdf;"),
    # rough dielectric
    ("Fresnel p-amplitude", "double rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);",
     "double rp = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);"),
    ("Fresnel Snell ratio", "double sin_t2 = sin_i2 / (eta * eta);", "double sin_t2 = sin_i2 / eta;"),
    ("refraction index inverted", "double a = c / eta - k;", "double a = c * eta - k;"),
    ("lobe choice inverted", "if (u3 < f) {", "if (u3 > f) {"),
    ("transmission Jacobian eta^2", "return (1.0 - f) * dv * eta * eta * std::fabs(co) / (den * den);",
     "return (1.0 - f) * dv * std::fabs(co) / (den * den);"),
    ("reflection Jacobian", "if (wo.z > 0.0) return f * dv / (4.0 * std::fabs(co));",
     "if (wo.z > 0.0) return f * dv / (2.0 * std::fabs(co));"),
    ("BTDF eta^2", "(wi.z * std::fabs(wo.z)) * eta * eta * (1.0 - f) *",
     "(wi.z * std::fabs(wo.z)) * (1.0 - f) *"),
    ("generalised half vector", "-(wi.x + eta * wo.x), -(wi.y + eta * wo.y),",
     "-(wi.x + wo.x / eta), -(wi.y + wo.y / eta),"),
    ("two-sided G1 side test", "if (!(dot(v, wm) / v.z > 0.0)) return 0.0;",
     "if (!(dot(v, wm) > 0.0)) return 0.0;"),
    ("dielectric G2 uncorrelated", "if (!(den > 0.0)) return 0.0;\n    return gi * go / den;",
     "if (!(den > 0.0)) return 0.0;\n    return gi * go;"),
    ("dielectric stream word", "*u3 = word_to_unit(w[2]);", "*u3 = word_to_unit(w[3]);"),
]


def _run_mutant(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not unique in oracle.cpp"
    path = os.path.join(tmp, name.replace(" ", "_"))
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "oracle.cpp"), "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(path, "liboracle.so")
    subprocess.run(["g++", "-O2", "-std=gnu++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
                    os.path.join(path, "oracle.cpp"), "-o", lib, "-lquadmath"], check=True)
    env = dict(os.environ, CAPVNDF_ORACLE_LIB=lib, CAPVNDF_ORACLE_THREADS="1",
               OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       timeout=600)
    return name, r.returncode, r.stdout.decode(errors="replace")[-2000:]


def test_every_mutant_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        workers = max(1, min(8, os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            results = list(ex.map(lambda m: _run_mutant(*m, tmp), MUTANTS))
    survivors = [name for name, rc, _ in results if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
    # every run failed in a test, not by crashing the collection
    for name, rc, out in results:
        assert rc == 1, f"{name}: pytest exited with {rc}:\n{out}"
