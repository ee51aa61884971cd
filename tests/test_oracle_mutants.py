"""Mutation check of the oracle's pins.

Each case copies oracle.c, plants one plausible mistake (a dropped term, a
wrong sign, index or constant, a transposed operand), builds the copy on the
CPU and runs the fast pins of test_oracle_pins against it: at least one pin
must fail.  The planted mistakes live only in these temporary copies.
"""
import inspect
import os
import shutil
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "philox_mul_swapped": ("(uint64_t)0xD2511F53u * (uint64_t)c[0]", "(uint64_t)0xCD9E8D57u * (uint64_t)c[0]"),
    "philox_no_key_bump": ("k[0] += 0x9E3779B9u;", "k[0] += 0u;"),
    "u24_wrong_shift": ("(double)(w >> 8) * 0x1p-24", "(double)(w >> 9) * 0x1p-24"),
    "shift_not_centred": ("s[k] = orc_u24(w[k]) - 0.5;", "s[k] = orc_u24(w[k]);"),
    "stream_dropped_h": ("double xe = fma(h, v[i], x[i]);", "double xe = v[i] + x[i];"),
    "stream_sign": ("double ye = fma(h, v[n + i], x[n + i]);", "double ye = fma(-h, v[n + i], x[n + i]);"),
    "wrap_wrong_branch": ("    x = x + L;\n  } else if (x >= L) {", "    x = x - L;\n  } else if (x >= L) {"),
    "wrap_far_collapses": ("      x = x - L * floor(x / L);", "      x = 0.0;"),
    "wrap_far_truncates": ("      x = x - L * floor(x / L);", "      x = x - L * trunc(x / L);"),
    "bounce_keeps_vx": ("v[i] = 2.0 * uw - v[i];", "v[i] = 2.0 * uw + v[i];"),
    "wall_frame_ignored": ("xe = xe - tr2 * (v[i] - uw);", "xe = xe - tr2 * v[i];"),
    "wall_velocity_sign": ("double uw = zw == 0.0 ? -p->uwall : p->uwall;",
                           "double uw = zw == 0.0 ? p->uwall : -p->uwall;"),
    "slip_mirrors_all": ("        if (p->slip) {\n          ze = ze - tr2 * vz;\n        } else {",
                         "        if (0) {\n          ze = ze - tr2 * vz;\n        } else {"),
    "slip_keeps_phantoms": ("if (p->walls && !p->slip) {", "if (p->walls) {"),
    "phantom_wall_velocity": ("for (int32_t q = 0; q < np; ++q) vp[3 * q] = vp[3 * q] + uw;",
                              "for (int32_t q = 0; q < np; ++q) vp[3 * q] = vp[3 * q] - uw;"),
    "bounce_mirror_factor": ("double tr2 = 2.0 * ((ze - zw) / vz);", "double tr2 = 1.0 * ((ze - zw) / vz);"),
    "keys_truncate": ("c[k] = (int64_t)floor(y);", "c[k] = (int64_t)y;"),
    "keys_y_fastest": ("key[i] = (uint32_t)((c[2] * p->L[1] + c[1]) * p->L[0] + c[0]);",
                       "key[i] = (uint32_t)((c[2] * p->L[0] + c[0]) * p->L[1] + c[1]);"),
    "sort_unstable": ("perm[offset[c] + count[c]] = (uint32_t)i;",
                      "perm[offset[c + 1] - 1 - count[c]] = (uint32_t)i;"),
    "rotate_sign": ("out[k] = ca * u[k] + sa * cr[k] + f * n[k];", "out[k] = ca * u[k] - sa * cr[k] + f * n[k];"),
    "rotate_dropped_parallel": ("out[k] = ca * u[k] + sa * cr[k] + f * n[k];", "out[k] = ca * u[k] + sa * cr[k];"),
    "cross_transposed": ("double cr[3] = {n[1] * u[2] - n[2] * u[1],", "double cr[3] = {n[2] * u[1] - n[1] * u[2],"),
    "vcm_wrong_mass": ("double M = (double)ntot * m;", "double M = (double)(ntot + 1) * m;"),
    "vcm_ignores_phantoms": ("double M = (double)ntot * m;", "double M = (double)nf * m;"),
    "kappa_missing_two": ("kappa = sqrt((2.0 * Ek) / K);", "kappa = sqrt(Ek / K);"),
    "gamma_shape_off": ("double d = shape - 1.0 / 3.0;", "double d = shape;"),
    "gamma_wrong_test": ("if (lhs < rhs) {", "if (lhs > rhs) {"),
    "dof_wrong": ("1.5 * (double)(ntot - 1)", "1.5 * (double)ntot"),
    "axis_not_uniform": ("double z = 1.0 - 2.0 * u1;", "double z = 1.0 - 2.0 * u1 * u1;"),
    "phantom_rate": ("double lam = p->density * fw;", "double lam = p->density;"),
    "phantom_variance": ("double sd = sqrt(p->kT / p->mass);", "double sd = p->kT / p->mass;"),
    "wall_fraction_bottom": ("    if (cz == 0) return sz;", "    if (cz == 0) return 1.0 - sz;"),
    "temperature_dof": ("nval(&K) / (3.0 * (double)(n - 1))", "nval(&K) / (3.0 * (double)n)"),
    "energy_half": ("nadd(&E, 0.5 * m * e);", "nadd(&E, m * e);"),
    "amc_omega_sign": ("om[k] = dk / det;", "om[k] = -dk / det;"),
    "amc_inertia_no_r2": ("(a == c ? r2 : 0.0) - r[a] * r[c]", "0.0 - r[a] * r[c]"),
    "amc_about_corner": ("for (int k = 0; k < 3; ++k) rc[k] = sum_val(&rs[k]) / (double)nf;",
                         "for (int k = 0; k < 3; ++k) rc[k] = 0.0;"),
    "amc_pair_factor": ("om[k] = dL[k] / (m * d2 / 2.0);", "om[k] = dL[k] / (m * d2);"),
    "amc_torque_post": ("u[k] = v0[k * n + i] - V[k];", "u[k] = v[k * n + i] - V[k];"),
    "amc_mbs_pre_energy": ("if (have_ek && K2 > 0.0) kappa = sqrt((2.0 * Ek) / K2);",
                           "if (have_ek && K2 > 0.0) kappa = sqrt((2.0 * Ek) / K);"),
    "amc_mbs_scaled_twice": ("const double kr = p->amc ? 1.0 : kappa;", "const double kr = kappa;"),
    "le_offset_time": ("double d = le_offset(p, t + 1);\n        if (ze >= Lz) {",
                       "double d = le_offset(p, t);\n        if (ze >= Lz) {"),
    "le_stream_sign": ("          xe = xe - d;", "          xe = xe + d;"),
    "le_stream_velocity": ("          v[i] = v[i] - p->le_u;\n        } else {",
                           "          v[i] = v[i] + p->le_u;\n        } else {"),
    "le_keys_image_sign": ("double xi = c[2] >= p->L[2] ? x[i] - d : x[i] + d;",
                           "double xi = c[2] >= p->L[2] ? x[i] + d : x[i] - d;"),
    "le_frame_not_restored": ("if (side < 0) v[i] = v[i] + p->le_u;", "if (side < 0) v[i] = v[i];"),
    "le_no_collision_frame": ("const int le = p->le_u != 0.0 && ntot >= 2;", "const int le = 0;"),
    "le_amc_torque_lab_frame": ("if (v0 && side < 0) v0[i] = v0[i] - p->le_u;",
                                "if (0) v0[i] = v0[i] - p->le_u;"),
    "le_amc_positions_unmapped": ("      if (side < 0) xa[i] = x[i] - d;", "      if (side < 0) xa[i] = x[i];"),
    "fixed_rounds_terms": ("a->s += (__int128)(x * 0x1p80);", "a->s += (__int128)nearbyint(x * 0x1p80);"),
    "fixed_scale_back": ("(double)a->s * 0x1p-80", "(double)a->s * 0x1p-79"),
    "fixed_range": ("} else if (fabs(x) < 0x1p37) {", "} else if (fabs(x) < 0x1p60) {"),
}

FAST_PINS = [
    "test_uniform_conversions", "test_shift_grid_and_uniformity", "test_stream_wrap_corner",
    "test_stream_wraps_far_outside",
    "test_stream_exact_single_rounding", "test_bounce_back_walls", "test_keys_exact_floor",
    "test_counting_sort_matches_numpy", "test_rotation_matches_scipy", "test_cell_sums_against_fsum",
    "test_collision_is_rotation_of_relative_velocity", "test_per_cell_momentum_and_energy_conservation",
    "test_special_angles", "test_axis_uniform_on_sphere", "test_gamma_sampler_distribution",
    "test_mbs_sets_cell_energy_to_drawn_value", "test_phantoms_enter_cell_sums",
    "test_phantom_count_and_velocity_laws", "test_wall_fraction_geometry",
    "test_observables_against_fsum", "test_reorder_is_gather", "test_philox_matches_rocrand",
    "test_amc_conserves_angular_momentum", "test_amc_correction_is_rigid_rotation",
    "test_amc_alpha_zero_is_identity", "test_amc_refused_with_walls", "test_amc_with_thermostat",
    "test_amc_with_slip_walls_conserves_angular_momentum",
    "test_fixed_sums_exact", "test_fixed_sums_order_independent", "test_fixed_sums_range",
    "test_moving_wall_bounce_is_galilean", "test_slip_walls_reflect_specularly",
    "test_slip_walls_exert_no_tangential_force", "test_couette_profile",
    "test_lees_edwards_stream", "test_lees_edwards_keys_use_the_image",
    "test_lees_edwards_momentum_budget", "test_lees_edwards_shear_profile",
    "test_amc_lees_edwards_conserves_angular_momentum",
]

PARAMS = {"test_keys_exact_floor": [{"walls": False}, {"walls": True}],
          "test_collision_is_rotation_of_relative_velocity": [{"mbs": False}, {"mbs": True}],
          "test_gamma_sampler_distribution": [{"shape": 3.0}, {"shape": 13.5}],
          "test_amc_conserves_angular_momentum": [{"L": (6, 6, 6), "density": 10.0},
                                                  {"L": (8, 8, 8), "density": 1.5}],
          "test_fixed_sums_order_independent": [{"amc": False}, {"amc": True}],
          "test_fixed_sums_exact": [{"vscale": 1.0}, {"vscale": 1e-13}]}


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand.cpp")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def caught_by(orc, rocrand_exe):
    for name in FAST_PINS:
        fn = getattr(pins, name)
        for extra in PARAMS.get(name, [{}]):
            kwargs = dict(extra)
            sig = inspect.signature(fn).parameters
            if "orc" in sig:
                kwargs["orc"] = orc
            if "rocrand_philox" in sig:
                if rocrand_exe is None:
                    continue
                kwargs["rocrand_philox"] = rocrand_exe
            try:
                fn(**kwargs)
            except (AssertionError, ValueError, FloatingPointError):
                return name
    return None


def test_unmutated_oracle_passes_fast_pins(rocrand_exe):
    assert caught_by(oracle, rocrand_exe) is None


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(mutant, tmp_path, rocrand_exe):
    old, new = MUTANTS[mutant]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {old}"
    mut_src = tmp_path / "oracle_mut.c"
    mut_src.write_text(src.replace(old, new, 1))
    so = str(tmp_path / "liboracle_mut.so")
    oracle.build(out=so, src=str(mut_src))
    with oracle.use_library(so):
        name = caught_by(oracle, rocrand_exe)
    assert name is not None, f"no pin caught mutant {mutant}"
    print(f"{mutant}: caught by {name}")
