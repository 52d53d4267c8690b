"""The oracle's pins must catch plausible mistakes: each case below plants one
mistake in a copy of the oracle source (on the CPU), rebuilds it, and requires
the named pin tests to fail against it."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "agal_oracle.c")

MUTANTS = [
    ("sat drops the face-normal axis",
     "if (s > r || s < -r) return 0;", "(void)s; (void)r;",
     "test_sat_3d_vs_exact_clipping"),
    ("sat edge axis with a flipped component",
     "else { iu = 0; iv = 1; au = -e[1]; av = e[0]; }", "else { iu = 0; iv = 1; au = e[1]; av = e[0]; }",
     "test_sat_3d_vs_exact_clipping"),
    ("2D sat with a transposed normal",
     "float Nx = -(Bv[1] - A[1]);\n    float Ny = Bv[0] - A[0];",
     "float Nx = Bv[0] - A[0];\n    float Ny = -(Bv[1] - A[1]);",
     "test_sat_2d_vs_exact_clipping"),
    ("bins linearised y-fastest",
     "bn->count[((int64_t)z * B + y) * B + x] += 1;", "bn->count[((int64_t)z * B + x) * B + y] += 1;",
     "test_bins_exact_circle or test_bins_exact_sphere_nondyadic_domain"),
    ("bin range upper end from the minimum",
     "hi_i[a] = bin_index(mx,", "hi_i[a] = bin_index(mn,",
     "test_bins_exact_circle or test_bins_exact_sphere_nondyadic_domain"),
    ("segment-triangle accepts v < 0",
     "if (v < 0.0 || u + v > 1.0) return 0;", "if (u + v > 1.0) return 0;",
     "test_links_exact_random_triangles"),
    ("segment-triangle t with the wrong sign",
     "double t = dot3(E2, Qv) / det;", "double t = -dot3(E2, Qv) / det;",
     "test_links_exact_random_triangles"),
    ("segment-segment with a transposed cross product",
     "double s = (w[0] * Dv[1] - w[1] * Dv[0]) / den;", "double s = (w[1] * Dv[0] - w[0] * Dv[1]) / den;",
     "test_links_exact_random_segments"),
    ("ties resolved to the highest face id",
     "if (t < best || (t == best && f < bf)) { best = t; bf = f; }",
     "if (t < best || (t == best && f > bf)) { best = t; bf = f; }",
     "test_links_closed_form_box"),
    ("ripple ignores diagonal neighbours",
     "if (!dx && !dy && !dz) continue;", "if (!dx && !dy && !dz) continue;\n                            if (dx && dy) continue;",
     "test_balance_and_structure or test_balance_is_minimal_closure"),
    ("cell centre shifted by half a cell",
     "(float)(2 * g + 1) * (0.5f * fo->dx[level][a])", "(float)(2 * g) * (0.5f * fo->dx[level][a])",
     "test_flags_closed_form_box_body"),
    ("every pass tested with the first level's distance",
     "cell_flag(fo, coords, F, bn, m, fo->d[l], &fo->tests[l])", "cell_flag(fo, coords, F, bn, m, fo->d[0], &fo->tests[l])",
     "test_flags_closed_form_box_body"),
    ("child coordinates with swapped bits",
     "ch.c[0] = 2 * b->c[0] + (ci & 1);", "ch.c[0] = 2 * b->c[0] + ((ci >> 1) & 1);",
     "test_flags_closed_form_box_body or test_links_closed_form_box"),
    ("adjoint barycentric weights permuted",
     "lam[0] = 1.0 - u - v; lam[1] = u; lam[2] = v;", "lam[0] = u; lam[1] = 1.0 - u - v; lam[2] = v;",
     "test_adjoint_horizontal_plane_closed_form or test_adjoint_matches_finite_differences"),
    ("adjoint with the normal of the wrong orientation in the numerator only",
     "grad[vk * dim + a] += wi * lam[k] * nrm[a] / den;", "grad[vk * dim + a] -= wi * lam[k] * nrm[a] / den;",
     "test_adjoint_horizontal_plane_closed_form or test_adjoint_matches_finite_differences"),
    ("2D adjoint with the segment weights swapped",
     "lam[0] = 1.0 - s; lam[1] = s;", "lam[0] = s; lam[1] = 1.0 - s;",
     "test_adjoint_horizontal_segment_closed_form or test_adjoint_2d_matches_finite_differences"),
    ("2D adjoint with a transposed segment normal",
     "n[0] = -(p[3] - p[1]);\n        n[1] = p[2] - p[0];", "n[0] = p[2] - p[0];\n        n[1] = -(p[3] - p[1]);",
     "test_adjoint_horizontal_segment_closed_form or test_adjoint_2d_matches_finite_differences"),
    ("near decision drops the face interior",
     "return hh * hh <= R2 * nn;", "return 0 && hh * hh <= R2 * nn;",
     "test_near_l2_f32_closed_boundary_dyadic or test_near_l2_f32_agrees_with_distance_off_the_boundary"),
    ("near decision with the edge-interior cross product from the wrong vector",
     "cross3f(e, w, c);\n        cc = dot3f(c, c);", "cross3f(e, p, c);\n        cc = dot3f(c, c);",
     "test_near_l2_f32_closed_boundary_dyadic or test_near_l2_f32_agrees_with_distance_off_the_boundary"),
    ("distance: segment parameter not clamped at the far end",
     "if (s > 1.0) s = 1.0;", "(void)0;",
     "test_face_distance_vs_numerical_minimisation"),
    ("own bin taken from the lower corner of the query box",
     "ix[a] = bin_index(m[a], bn->lo[a], bn->s[a], bn->B);", "ix[a] = bin_index(m[a] - R, bn->lo[a], bn->s[a], bn->B);",
     "test_own_bin_flags_and_propagation_brute_force"),
    ("propagation marks in one sweep (a step can run on through blocks it just marked)",
     "if (nb && nb->pass_mark == 0) nb->pass_mark = 4;", "if (nb && nb->pass_mark == 0) { nb->pass_mark = 3; nb->mark = 3; }",
     "test_own_bin_flags_and_propagation_brute_force"),
    ("one propagation step too few",
     "return 1 + (int)floorf(fo->d[l] / (4.0f * dxm));", "return (int)floorf(fo->d[l] / (4.0f * dxm));",
     "test_own_bin_flags_and_propagation_brute_force"),
    ("2D classification with the segment normal reversed",
     "nrm[0] = e1;\n                nrm[1] = -e0;", "nrm[0] = -e1;\n                nrm[1] = e0;",
     "test_classify_circle_matches_winding_number"),
    ("3D classification with a transposed cross-product component",
     "nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];", "nrm[1] = e1[0] * e2[2] - e1[2] * e2[0];",
     "test_classify_3d_matches_winding_number"),
    ("classification never reports disagreeing links",
     "cls[k] = (uint8_t)(enter && leave ? 3", "cls[k] = (uint8_t)(0 ? 3",
     "test_classify_dyadic_box_exact"),
    ("classification reads the lattice one direction off",
     "double sgn = ((double)c[3 * i] * nrm[0] + (double)c[3 * i + 1] * nrm[1]) + (double)c[3 * i + 2] * nrm[2];",
     "double sgn = ((double)c[3 * i - 3] * nrm[0] + (double)c[3 * i - 2] * nrm[1]) + (double)c[3 * i - 1] * nrm[2];",
     "test_classify_3d_matches_winding_number or test_classify_circle_matches_winding_number"),
    ("re-adaptation with refined and coarsened swapped",
     "state[i] = 2;\n        else if (!old_leaf[j] && new_leaf[i]) state[i] = 3;",
     "state[i] = 3;\n        else if (!old_leaf[j] && new_leaf[i]) state[i] = 2;",
     "test_diff_matches_brute_force"),
    ("re-adaptation looks removed blocks up in the old level",
     "removed[j] = key_search(new_keys, n_new, old_keys[j]) < 0 ? 1 : 0;",
     "removed[j] = key_search(old_keys, n_old, old_keys[j]) < 0 ? 1 : 0;",
     "test_diff_family_structure"),
    ("re-adaptation maps a kept block to its own index",
     "old_index[i] = (int32_t)j;", "old_index[i] = j < 0 ? -1 : (int32_t)i;",
     "test_diff_family_structure or test_diff_matches_brute_force"),
    ("sampled binning fans its segments towards the wrong vertex",
     "g[x] = fc[6 + x] - q[x];", "g[x] = fc[x] - q[x];",
     "test_assigned_bins_meet_the_face_and_hold_its_vertices or test_spacing_above_the_face_samples_its_vertices_only"),
    ("sampled binning one subdivision too coarse",
     "while (k < ORC_DISC_KMAX && !(s <= ldexpf(spacing, k))) ++k;",
     "while (k < ORC_DISC_KMAX && !(s <= ldexpf(spacing, k + 1))) ++k;",
     "test_segments_cover_every_bin_they_cross_by_more_than_the_spacing"),
    ("sampled binning stops half way along the first edge",
     "float t = ldexpf((float)j, -k1);", "float t = ldexpf((float)j, -k1 - 1);",
     "test_assigned_bins_meet_the_face_and_hold_its_vertices or test_spacing_above_the_face_samples_its_vertices_only"),
    ("sampled binning with the bin index transposed",
     "int64_t bb = ((int64_t)ix[2] * B + ix[1]) * B + ix[0];", "int64_t bb = ((int64_t)ix[2] * B + ix[0]) * B + ix[1];",
     "test_assigned_bins_meet_the_face_and_hold_its_vertices"),
]


@pytest.mark.parametrize("name,old,new,tests", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, tests):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = src.replace(old, new)
    cpath = tmp_path / "mut.c"
    cpath.write_text(mutated)
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", str(cpath), "-o", str(lib), "-lm"])
    env = dict(os.environ, AGAL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"), os.path.join(HERE, "test_oracle_own_bin.py"),
                        os.path.join(HERE, "test_oracle_classify.py"), os.path.join(HERE, "test_oracle_readapt.py"),
                        os.path.join(HERE, "test_oracle_discrete_bins.py"),
                        "-k", tests],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
