"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's source (CPU only),
builds it, and runs the oracle's pin suite against that copy, which must then
fail.  The mistakes cover every step: keys, tree, moments, walk, the Green's
function derivatives, eqs. 2-4, the correction of eq. 7 (prefactor and sign)
the near field, and the learned pair selection (rounding, logarithm, features,
labels, gradient, gating).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

CORE_PINS = ["tests/test_oracle_greens.py", "tests/test_oracle_tree.py", "tests/test_oracle_moments.py",
             "tests/test_oracle_pair.py", "tests/test_oracle_solve.py"]
FIELD_PINS = ["tests/test_oracle_field_walk.py"]
LEARNED_PINS = ["tests/test_oracle_learned.py"]


def pins_for(name):
    """The pin files that cover the step a mistake is planted in (the others
    cannot see it and only cost time)."""
    if name.startswith("field_"):
        return FIELD_PINS
    if name.startswith("multipole_"):
        return ["tests/test_oracle_multipole.py"]
    if name.split("_")[0] in ("learned", "label", "grad", "plog2", "bf16", "feature"):
        return LEARNED_PINS
    if name.startswith("soft_"):
        return ["tests/test_oracle_softening.py"]
    if name.startswith("order_"):
        return ["tests/test_oracle_order.py"]
    return CORE_PINS

MUTATIONS = {
    "order_correction_sign": ("    gp.Fc[k] = -s;", "    gp.Fc[k] = s;"),
    "order_drop_quadrupole_pair": ("      if (n == 1 || P - n == 1) continue;",
                                   "      if (n == 1 || P - n == 1 || (n > 0 && n < P)) continue;"),
    "order_source_sign": ("      double sb = (nb % 2) ? -1.0 : 1.0;", "      double sb = 1.0;"),
    "order_mirror_sign": ("    if (kMI.order[al] % 2) gp.Lb[al] = -gp.Lb[al];", ""),
    "order_pairing_count": ("            ways /= power(2.0, b[i]);", "            ways /= 1.0;"),
    "correction_prefactor_half": ("pt.Fc[i] = -(1.0 / 6.0) * s;", "pt.Fc[i] = -(0.5) * s;"),
    "correction_sign": ("pt.Fc[i] = -(1.0 / 6.0) * s;", "pt.Fc[i] = (1.0 / 6.0) * s;"),
    "separation_sign": ("double R[3] = {A.Z[0] - B.Z[0], A.Z[1] - B.Z[1], A.Z[2] - B.Z[2]};\n  if (eps2 > 0.0)",
                        "double R[3] = {B.Z[0] - A.Z[0], B.Z[1] - A.Z[1], B.Z[2] - A.Z[2]};\n  if (eps2 > 0.0)"),
    "order_separation_sign": ("double R[3] = {A.Z[0] - B.Z[0], A.Z[1] - B.Z[1], A.Z[2] - B.Z[2]};\n  std::vector<double> D;",
                              "double R[3] = {B.Z[0] - A.Z[0], B.Z[1] - A.Z[1], B.Z[2] - A.Z[2]};\n  std::vector<double> D;"),
    "eq3_quadrupole_half_dropped": ("    c0 += 0.5 * q;", "    c0 += q;"),
    "eq4_cubic_sign": ("out[i] = -(c0 + c1 - 0.5 * c2);", "out[i] = -(c0 + c1 + 0.5 * c2);"),
    "d3_coefficient": ("(15.0 * R[i] * R[j] * R[k] -", "(5.0 * R[i] * R[j] * R[k] -"),
    "d4_coefficient": ("double t4 = -105.0 *", "double t4 = -15.0 *"),
    "d4prime_extra_term": ("g.D4p[i][j][k][l] = p2 + t0;", "g.D4p[i][j][k][l] = p2 + t0 + t4;"),
    "quadrupole_without_mass": ("mo.M2[i][j] += mu * xv[i] * xv[j];", "mo.M2[i][j] += xv[i] * xv[j];"),
    "octupole_transposed": ("mo.M3[i][j][k] += mu * xv[i] * xv[j] * xv[k];",
                            "mo.M3[i][j][k] += mu * xv[i] * xv[j] * xv[j];"),
    "criterion_one_radius": ("double rhs = (A.Rmax + B.Rmax) / t.theta;", "double rhs = (A.Rmax) / t.theta;"),
    "criterion_stricter": ("double rhs = (A.Rmax + B.Rmax) / t.theta;", "double rhs = 1.25 * (A.Rmax + B.Rmax) / t.theta;"),
    "key_bits_swapped": ("key |= ((q[0] >> b) & 1) << (3 * b + 2);", "key |= ((q[0] >> b) & 1) << (3 * b + 1);"),
    "split_at_ncrit": ("if (!(cur.count > n_crit && lev < max_level)) continue;",
                       "if (!(cur.count >= n_crit && lev < max_level)) continue;"),
    "near_field_no_reaction": ("gx[j] -= t->m[i] * dx / r3;", "gx[j] -= 0.0 * dx / r3;"),
    "potential_quadratic_half": ("return p + 0.5 * s2 + (1.0 / 6.0) * s3;", "return p + s2 + (1.0 / 6.0) * s3;"),
    "field_one_sided": ("return r6 * (B.M * B.M) <= (wa * wa) * d10 && r6 * (A.M * A.M) <= (wb * wb) * d10;",
                        "return r6 * (B.M * B.M) <= (wa * wa) * d10;"),
    "field_cube_not_sixth": ("double r6 = (r2 * r2) * r2;", "double r6 = r2 * r2;"),
    "field_scale_no_floor": ("std::max(gmin[ci], 0.1 * (gsum[ci] / (double)t->cells[ci].count))",
                             "std::max(gmin[ci], 1.0 * (gsum[ci] / (double)t->cells[ci].count))"),
    "learned_gate_low": ("double lo = 0.25 * t.eps, hi = 2.0 * t.eps;", "double lo = 0.5 * t.eps, hi = 2.0 * t.eps;"),
    "learned_small_pairs_accept_all": ("if (t.cells[a].count * t.cells[b].count < t.min_work) return plain;",
                                       "if (t.cells[a].count * t.cells[b].count < t.min_work) return true;"),
    "learned_one_cell": ("bool plain = ea <= (t.eps * sa) * d6 && eb <= (t.eps * sb) * d6;",
                         "bool plain = ea <= (t.eps * sa) * d6;"),
    "learned_rho_sign": ("return mlp_infer(P, f) <= (float)(-plog2(rho));",
                         "return mlp_infer(P, f) <= (float)(plog2(rho));"),
    "label_mean_not_max": ("E = std::max(E, std::sqrt((ex * ex + ey * ey) + ez * ez));",
                           "E += std::sqrt((ex * ex + ey * ey) + ez * ez) / (double)ns;"),
    "label_estimate_own_moments": ("int k2s = norm_level(traceless_norm2(MS), MS.M, MS.Rmax, 2);",
                                   "int k2s = norm_level(traceless_norm2(MT), MT.M, MT.Rmax, 2);"),
    "grad_no_relu_mask": ("double dz1 = z1[j] > 0.0 ? dh : 0.0;", "double dz1 = dh;"),
    "plog2_off_by_one": ("return (double)(e - 1) + (2.0 * m - 1.0);", "return (double)(e) + (2.0 * m - 1.0);"),
    "bf16_truncates": ("u += 0x7FFFu + ((u >> 16) & 1u);", "u += 0u;"),
    "feature_antisymmetric": ("f[3] = (float)((double)std::abs(k2a - k2b) / 128.0);",
                              "f[3] = (float)((double)(k2a - k2b) / 128.0);"),
    "multipole_one_sided": ("return ea <= (t.eps * t.fscale[a]) * d6 && eb <= (t.eps * t.fscale[b]) * d6;",
                            "return ea <= (t.eps * t.fscale[a]) * d6;"),
    "multipole_stricter": ("return ea <= (t.eps * t.fscale[a]) * d6 && eb <= (t.eps * t.fscale[b]) * d6;",
                           "return 1.25 * ea <= (t.eps * t.fscale[a]) * d6 && 1.25 * eb <= (t.eps * t.fscale[b]) * d6;"),
    "multipole_power_of_d": ("    double d6 = (d2 * d2) * d2;", "    double d6 = (d2 * d2) * d;"),
    "multipole_extents_swapped": ("double ea = multipole_bracket(A.Rmax, B.Rmax, t.k2[b], t.k3[b], d) * B.M;",
                                  "double ea = multipole_bracket(B.Rmax, A.Rmax, t.k2[b], t.k3[b], d) * B.M;"),
    "multipole_octupole_not_traceless": ("double w = mo.M3[i][j][k] - (v[i] * kdelta(j, k) + v[j] * kdelta(i, k) + v[k] * kdelta(i, j)) / 5.0;",
                                         "double w = mo.M3[i][j][k];"),
    "multipole_no_target_truncation": ("kMw1 * (rt2 * rt);", "0.0 * (rt2 * rt);"),
    "multipole_quadrupole_not_traceless": ("double v = mo.M2[i][j] - (i == j ? tr / 3.0 : 0.0);",
                                           "double v = mo.M2[i][j];"),
    "multipole_level_truncates": ("double k = std::floor(kMq * (norm / den) + 0.5);",
                                  "double k = std::floor(kMq * (norm / den));"),
    "multipole_source_terms_swapped": ("double Q = kMw4 * (rs2 * rs2) + kMw5 * (rt2 * rt2);",
                                       "double Q = kMw5 * (rs2 * rs2) + kMw4 * (rt2 * rt2);"),
    "soft_f3_coefficient": ("double f3 = -5.0 * f2 / s;", "double f3 = -3.0 * f2 / s;"),
    "soft_direct_unsoftened": ("      double s2 = r2 + eps2;", "      double s2 = r2;"),
    "soft_D4_missing_terms": ("g.D4[i][j][k][l] = f2 * dd + f3 * (di + dr) + f4 * R[i] * R[j] * R[k] * R[l];",
                              "g.D4[i][j][k][l] = f2 * dd + f3 * di + f4 * R[i] * R[j] * R[k] * R[l];"),
    "self_walk_skips_pairs": ("for (int32_t b = a + 1; b < C.child0 + C.nchild; ++b) walk_pair(t, a, b);",
                              "for (int32_t b = a + 2; b < C.child0 + C.nchild; ++b) walk_pair(t, a, b);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old}"
    mut = tmp_path / "oracle_mut.cpp"
    mut.write_text(src.replace(old, new))
    inc = os.path.join(ROOT, "oracle")
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c++17",
                    "-I", inc, str(mut), "-o", str(so)], check=True)
    env = dict(os.environ, AMFMM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + pins_for(name), cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
