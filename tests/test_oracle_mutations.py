"""The oracle's boundary pins are strong enough to catch plausible mistakes.

Each case copies the oracle source, plants one mistake in a boundary formula
(Sec. II.C.1 Grad target values and fresh-node fill, Sec. II.C.2 wall stress),
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

# (name, original text, planted text, pin, pin arguments)
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
]

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    import oracle
    oracle._SRC = {src!r}
    oracle._LIB = {lib!r}
    oracle.build(force=True)
    import test_oracle_domain as T
    try:
        getattr(T, {pin!r})(oracle, *{args!r})
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
