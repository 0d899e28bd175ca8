"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies the oracle source, plants one mistake in a boundary formula
(Sec. II.C.1 Grad target values and fresh-node fill, Sec. II.C.2 wall stress,
surface meshes) or in the multiphase step (Sec. III.B),
builds the copy in a temporary directory and runs one domain pin against it in
a child process; the pin must fail.  Nothing here touches the GPU path.
"""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, original text, planted text, pin ("module:function", or a function of
# test_oracle_domain), pin arguments)
CASES = [
    # Wall stress extrapolated from the far probe instead of to the wall.
    ("stress_extrapolation_reversed",
     "(2.0 * s1[3 * a + b] - s2[3 * a + b]) * nv[b]",
     "(2.0 * s2[3 * a + b] - s1[3 * a + b]) * nv[b]",
     "test_poiseuille_channel_inlet_outlet_walls", ()),
    # Viscous stress without the (1 - beta) factor.
    ("stress_without_one_minus_beta",
     "-(1.0 - beta) * pi1", "-pi1",
     "test_poiseuille_channel_inlet_outlet_walls", ()),
    # Fresh nodes refilled at rest instead of at the body velocity.
    ("fresh_node_at_rest",
     "body_velocity(d.body, D, p, t1, ub);", "ub[0] = ub[1] = ub[2] = 0.0;",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Wall-motion term of the target density with the wrong sign.
    ("target_density_motion_sign",
     "rho_t += Ax[Q - 1 - i] + 6.0 * L.w[i] * rho_n[n] * cu;",
     "rho_t += Ax[Q - 1 - i] - 6.0 * L.w[i] * rho_n[n] * cu;",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Quadratic interpolation weight of x + c_i with q and 1 - q exchanged.
    ("target_velocity_weight_q_swapped",
     "const double a1 = 2.0 * qq / (1.0 + qq);",
     "const double a1 = 2.0 * (1.0 - qq) / (1.0 + qq);",
     "test_couette_through_grad_walls", (0.25, 0.75)),
    # One-sided gradient through the wall point with the wall term's sign flipped.
    ("gradient_wall_term_sign",
     "g = -3.0 * w0 / ((1.0 + qq) * (2.0 + qq)) + u_n[3 * p1 + a] * (2.0 - qq) / (1.0 + qq) +",
     "g = 3.0 * w0 / ((1.0 + qq) * (2.0 + qq)) + u_n[3 * p1 + a] * (2.0 - qq) / (1.0 + qq) +",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Fresh node refilled at the reference density instead of its neighbours'.
    ("fresh_density_reference",
     "const double rb = cnt ? sum / cnt : 1.0;", "const double rb = 1.0;",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Fresh-node density summed instead of averaged.
    ("fresh_density_sum_not_mean",
     "const double rb = cnt ? sum / cnt : 1.0;", "const double rb = cnt ? sum : 1.0;",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Fresh-node density average over solid neighbours as well.
    ("fresh_density_includes_solid",
     "        if (d.solid[m]) continue;\n        sum += rho_n[m];", "        sum += rho_n[m];",
     "test_body_carried_by_uniform_flow_leaves_it_uniform", ()),
    # Linear target-velocity fallback with the wall and x + c_i weights exchanged.
    ("target_velocity_linear_fallback_weights",
     "for (int a = 0; a < 3; ++a) ui[a] = (uw[i][a] + qq * u_n[3 * m1 + a]) / (1.0 + qq);",
     "for (int a = 0; a < 3; ++a) ui[a] = (qq * uw[i][a] + u_n[3 * m1 + a]) / (1.0 + qq);",
     "test_target_velocity_linear_fallback_and_linear_wall_gradient", ()),
    # Target velocity at rest where no lattice neighbour along c_i is fluid.
    ("target_velocity_no_fluid_fallback",
     "      for (int a = 0; a < 3; ++a) ui[a] = uw[i][a];",
     "      for (int a = 0; a < 3; ++a) ui[a] = 0.0;",
     "test_target_single_row_between_two_cut_walls", ()),
    # Central difference without the factor 1/2.
    ("gradient_central_factor",
     "g = 0.5 * (u_n[3 * p1 + a] - u_n[3 * m1 + a]);",
     "g = (u_n[3 * p1 + a] - u_n[3 * m1 + a]);",
     "test_target_gradient_central_difference", ()),
    # Linear difference through the wall point without the spacing 1 + q.
    ("gradient_linear_wall_spacing",
     "g = (u_n[3 * p1 + a] - w0) / (1.0 + qq);", "g = (u_n[3 * p1 + a] - w0);",
     "test_target_velocity_linear_fallback_and_linear_wall_gradient", ()),
    # Two cut sides: central-difference spacing instead of the wall distance.
    ("gradient_two_sided_cut_spacing",
     "g = (uw[im][a] - uw[ip][a]) / (q[im] + q[ip]);", "g = 0.5 * (uw[im][a] - uw[ip][a]);",
     "test_target_single_row_between_two_cut_walls", ()),
    # Probe fallback searching the 3^D box only.
    ("probe_fallback_box_3",
     "    for (int dy = -2; dy <= 2; ++dy)\n      for (int dx = -2; dx <= 2; ++dx) {",
     "    for (int dy = -1; dy <= 1; ++dy)\n      for (int dx = -1; dx <= 1; ++dx) {",
     "test_poiseuille_channel_inlet_outlet_walls", ()),
    # Probe fallback with the maximum-norm distance.
    ("probe_fallback_max_norm",
     "for (int a = 0; a < D; ++a) r2 += (q[a] - p[a]) * (q[a] - p[a]);",
     "for (int a = 0; a < D; ++a) r2 = std::max(r2, std::fabs(q[a] - p[a]));",
     "test_probe_fallback_nearest_fluid_node_brute_force", (9,)),
    # Solid angle of a triangle without its factor 2 (winding number halved).
    ("mesh_solid_angle_half",
     "    sum += 2.0 * std::atan2(det, den);", "    sum += std::atan2(det, den);",
     "test_oracle_mesh:test_cube_mesh_solid_is_the_box", (False,)),
    # 2D winding with the cross and dot products exchanged.
    ("mesh_polygon_angle_swapped",
     "    sum += std::atan2(ax * by - ay * bx, ax * bx + ay * by);",
     "    sum += std::atan2(ax * bx + ay * by, ax * by - ay * bx);",
     "test_oracle_mesh:test_square_polygon_solid_is_the_square_2d", ()),
    # Mesh velocity interpolated with the second and third vertices exchanged.
    ("mesh_velocity_vertices_swapped",
     "        v[a] = l[0] * b.mvel[3 * i0 + a] + l[1] * b.mvel[3 * i1 + a] +",
     "        v[a] = l[0] * b.mvel[3 * i0 + a] + l[1] * b.mvel[3 * i2 + a] +",
     "test_oracle_mesh:test_rigid_motion_targets_exact_on_mesh", (27,)),
    # Closest point on the third edge with a sign error.
    ("mesh_closest_edge_sign",
     "      const double t = f > 0.0 ? clamp01((A + Dv - B - E) / f) : 0.0;",
     "      const double t = f > 0.0 ? clamp01((A - Dv - B - E) / f) : 0.0;",
     "test_oracle_mesh:test_mesh_velocity_at_closest_point_of_a_box", ()),
    # Closest point on the first edge unclamped.
    ("mesh_closest_edge_unclamped",
     "      const double s = A > 0.0 ? clamp01(-Dv / A) : 0.0;",
     "      const double s = A > 0.0 ? -Dv / A : 0.0;",
     "test_oracle_mesh:test_mesh_velocity_at_closest_point_of_a_box", ()),
    # Mesh solid test without the explicit surface rule.
    ("mesh_surface_not_solid",
     "      return std::fabs(D == 3 ? winding_3d(b, x) : winding_2d(b, x)) > 0.5 ||\n             mesh_dist2(b, D, x) <= 1e-24;",
     "      return std::fabs(D == 3 ? winding_3d(b, x) : winding_2d(b, x)) > 0.5;",
     "test_oracle_mesh:test_nodes_on_the_surface_are_solid", (9,)),
    # Korteweg term with the sign printed in the paper's reduced form.
    ("mp_kappa_sign",
     "2.0 * phi[n] * (3.0 * gphi[a]) + d.kappa * rho[n] * (3.0 * glap[a]) +",
     "2.0 * phi[n] * (3.0 * gphi[a]) - d.kappa * rho[n] * (3.0 * glap[a]) +",
     "test_oracle_multiphase:test_flat_interface_coexistence_matches_printed", (9,)),
    # phi gradient stencil without the 1 / cs^2 factor.
    ("mp_gradient_factor",
     "2.0 * phi[n] * (3.0 * gphi[a])", "2.0 * phi[n] * (1.0 * gphi[a])",
     "test_oracle_multiphase:test_phi_gradient_term_exact_on_linear_phi", (27,)),
    # Laplacian stencil with the factor 1 / cs^2 instead of 2 / cs^2.
    ("mp_laplacian_factor",
     "    lap[n] = 6.0 * s;", "    lap[n] = 3.0 * s;",
     "test_oracle_multiphase:test_korteweg_term_exact_on_cubic_density", (9,)),
    # Non-fluid neighbour read as zero density instead of the node's own.
    ("mp_solid_neighbour_zero",
     "      const double v = fluid_nb(x, i, &m) ? rho[m] : rho[n];",
     "      const double v = fluid_nb(x, i, &m) ? rho[m] : 0.0;",
     "test_oracle_multiphase:test_wetting_force_flat_wall_and_corner", (9,)),
    # Wetting sum over the fluid neighbours instead of the solid ones.
    ("mp_wetting_fluid_set",
     "        if (!fl) wet[a] += L.w[i] * L.c[i][a];",
     "        if (fl) wet[a] += L.w[i] * L.c[i][a];",
     "test_oracle_multiphase:test_wetting_force_at_a_body", ()),
    # EOS with one coefficient's sign flipped.
    ("mp_eos_coefficient",
     "                              4.139745482116095e-3,",
     "                              -4.139745482116095e-3,",
     "test_oracle_multiphase:test_flat_interface_coexistence_matches_printed", (9,)),
    # Stabiliser from the unshifted scalar product.
    ("mp_gamma_unshifted",
     "      a += ds[i] * dh[i] / feqs[i];\n      b += dh[i] * dh[i] / feqs[i];",
     "      a += ds[i] * dh[i] / feq[i];\n      b += dh[i] * dh[i] / feq[i];",
     "test_oracle_multiphase:test_shifted_gamma_minimises_shifted_entropy_norm", (27,)),
    # Multiphase wall fill without the bounce-back mass.
    ("mp_fill_unscaled",
     "          const double lam = (rho_t - sk) / sm;", "          const double lam = 1.0;",
     "test_oracle_multiphase:test_droplet_on_non_wetting_wall_keeps_its_mass", ()),
    # Exact difference method with half the velocity increment.
    ("mp_edm_half_increment",
     "    us[a] = u[a] + F[a] / rho;", "    us[a] = u[a] + 0.5 * F[a] / rho;",
     "test_oracle_multiphase:test_forced_step_keeps_mass_and_adds_force", (9,)),
]

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    import oracle
    oracle._SRC = {src!r}
    oracle._LIB = {lib!r}
    oracle.build(force=True)
    import importlib
    mod, _, fn = {pin!r}.rpartition(":")
    T = importlib.import_module(mod or "test_oracle_domain")
    try:
        getattr(T, fn)(oracle, *{args!r})
    except AssertionError:
        print("PIN FAILED")
        sys.exit(0)
    print("PIN PASSED")
""")


@pytest.mark.parametrize("name,orig,planted,pin,args", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_fails_a_pin(tmp_path, name, orig, planted, pin, args):
    src = open(oracle._SRC).read()
    assert src.count(orig) == 1, "the text to mutate must occur exactly once"
    msrc = tmp_path / ("mut_%s.cpp" % name)
    msrc.write_text(src.replace(orig, planted))
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), src=str(msrc),
                        lib=str(tmp_path / ("mut_%s.so" % name)), pin=pin, args=tuple(args))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "PIN FAILED" in r.stdout, "planted mistake %s was not caught by %s" % (name, pin)


# Planted mistakes in the Python parts of the oracle (the beam and the
# coupling): (module file, original text, planted text, pin module:function).
PY_CASES = [
    ("fsi_reference_pressure_as_load", "fsi.py",
     "tr = np.asarray(tr).reshape(-1, 2) + nrm / 3.0", "tr = np.asarray(tr).reshape(-1, 2)",
     "test_oracle_fsi:test_fluid_at_rest_leaves_the_beam_at_rest"),
    ("fsi_normal_inward", "fsi.py",
     "nrm.append(np.array([t[1], -t[0]]) / L)", "nrm.append(np.array([-t[1], t[0]]) / L)",
     "test_oracle_fsi:test_wet_edge_quadrature_of_the_undeformed_beam"),
    ("fem_tangent_without_geometric_term", "fem.py",
     "        dP = geo + mat", "        dP = mat",
     "test_oracle_fem:test_tangent_is_derivative_of_internal_force"),
    ("fem_green_strain_linearised", "fem.py",
     "        E = 0.5 * (np.einsum(\"egkI,egkJ->egIJ\", F, F) - np.eye(2))\n        trE",
     "        E = 0.5 * (G + np.swapaxes(G, -1, -2))\n        trE",
     "test_oracle_fem:test_csm3_tip_motion_matches_printed"),
]

PY_CHILD = textwrap.dedent("""
    import importlib.util, sys, types
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    import oracle
    spec = importlib.util.spec_from_file_location("oracle.{mod}", {path!r})
    m = importlib.util.module_from_spec(spec)
    sys.modules["oracle.{mod}"] = m
    spec.loader.exec_module(m)
    setattr(oracle, "{mod}", m)
    import importlib
    mod, _, fn = {pin!r}.rpartition(":")
    T = importlib.import_module(mod)
    import inspect
    f = getattr(T, fn)
    try:
        f(*([oracle] if "orc" in inspect.signature(f).parameters else []))
    except AssertionError:
        print("PIN FAILED")
        sys.exit(0)
    print("PIN PASSED")
""")


@pytest.mark.parametrize("name,fname,orig,planted,pin", PY_CASES, ids=[c[0] for c in PY_CASES])
def test_planted_mistake_in_python_oracle_fails_a_pin(tmp_path, name, fname, orig, planted, pin):
    src = open(os.path.join(ROOT, "oracle", fname)).read()
    assert src.count(orig) == 1, "the text to mutate must occur exactly once"
    p = tmp_path / fname
    p.write_text(src.replace(orig, planted))
    code = PY_CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), mod=fname[:-3],
                           path=str(p), pin=pin)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "PIN FAILED" in r.stdout, "planted mistake %s was not caught by %s" % (name, pin)
