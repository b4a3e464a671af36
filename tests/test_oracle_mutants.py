"""The oracle's pins have the power to catch plausible mistakes.

Each case below plants one mistake in a copy of the oracle's C source (on the
CPU, in a temporary directory), builds it, routes the oracle binding to it and
runs the pins: at least one pin must fail.  A mutant that every pin accepts
would be a part of the oracle that nothing independent fixes.
"""
import os
import tempfile

import pytest

import oracle

import test_oracle_pins as P
import test_oracle_strain_pins as S

# (name, text in the oracle source, replacement, pins expected to catch it)
MUTANTS = [
    ("bend X*X for X*Z", "c[4] * X * Z", "c[4] * X * X", ["poly2_bend"]),
    ("Z sign flipped", "Z = z - d->z_ref_um", "Z = d->z_ref_um - z", ["poly2_bend", "poly2_z_terms"]),
    ("strain at z_{n+1}", "oracle_strain_phase(d, j, step)", "oracle_strain_phase(d, j, step + 1)",
     ["poly2_bend", "poly2_z_terms"]),
    ("x0 dropped", "double x = d->x0_um + j * d->dx_um;", "double x = j * d->dx_um;",
     ["poly2_bend", "poly2_linear_x"]),
    ("c1 times Z", "c[1] * X", "c[1] * Z", ["poly2_linear_x"]),
    ("c2 times X", "c[2] * Z", "c[2] * X", ["poly2_z_terms"]),
    ("c5 Z for Z^2", "c[5] * Z * Z", "c[5] * Z", ["poly2_z_terms"]),
    ("c3 X*Z for X^2", "c[3] * X * X", "c[3] * X * Z", ["poly2_quadratic_x"]),
    ("c0 dropped", "u = c[0] + c[1] * X", "u = c[1] * X", ["poly2_z_terms"]),
    ("table transposed", "u_table[(size_t)n * d->nx + j]", "u_table[(size_t)j * d->nz + n]",
     ["table_orientation", "table_bend"]),
    ("dislocation 4(1-nu)", "X * Z / (2.0 * (1.0 - d->disl_nu) * r2)", "X * Z / (4.0 * (1.0 - d->disl_nu) * r2)",
     ["disl_vector_form", "disl_equilibrium"]),
    ("dislocation XZ term dropped", "if (r2 > 0) t += X * Z", "if (r2 < 0) t += X * Z",
     ["disl_vector_form", "disl_equilibrium"]),
    ("atan2 arguments swapped", "atan2(Z, X)", "atan2(X, Z)", ["disl_vector_form", "disl_equilibrium"]),
    ("dislocation winding reversed", "double t = atan2(Z, X);", "double t = -atan2(Z, X);",
     ["disl_vector_form", "disl_winding"]),
    ("evanescent growth", "exp(-sc.dzh * sqrt(p * p - 1.0))", "exp(sc.dzh * sqrt(p * p - 1.0))", ["evanescent"]),
    ("evanescent phase sign", "cexp(-I * sc.dzh * sc.c);\n            }\n            P /= (double)n;",
     "cexp(I * sc.dzh * sc.c);\n            }\n            P /= (double)n;", ["evanescent"]),
    ("3D evanescent growth", "P = exp(-dzh * sqrt(-r)) * cexp(-I * dzh * sc.c);",
     "P = exp(dzh * sqrt(-r)) * cexp(-I * dzh * sc.c);", ["evanescent_3d"]),
    ("3D evanescent threshold on qx only", "double r = 1.0 - px * px - qy * qy;", "double r = 1.0 - px * px;",
     ["evanescent_3d"]),
    ("strain sign on psi+", "psi_p[j] = sc.a0 * p + sc.ap * e * m;", "psi_p[j] = sc.a0 * p + sc.ap * conj(e) * m;",
     ["coupling_sign", "poly2_linear_x"]),
    ("a+ paired with chihb", "*ap = I * A * chih * off * E;", "*ap = I * A * chihb * off * E;",
     ["coupling_sign", "poly2_linear_x"]),
    ("split sub-steps all at z_n", "zoff[i] = acc;", "zoff[i] = 0.0;", ["poly2_bend_order2"]),
    # order 2 has a = (0, 1), so its heights equal the a_i themselves; order 4 does not
    ("split height a_i for the running sum", "zoff[i] = acc;", "zoff[i] = a[i];", ["split4_heights"]),
]

PINS = dict(S.PINS)
PINS["disl_winding"] = P.test_dislocation_phase_winds_by_h_dot_b
PINS["split4_heights"] = lambda: P.test_split_sub_steps_sample_the_strain_at_their_own_height(4)


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory(prefix="oracle_mutants_") as d:
        yield d


def test_every_pin_passes_on_the_oracle():
    for name, fn in PINS.items():
        fn()


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(workdir, name, old, new, pins):
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation site not found exactly once: %r" % old
    path = os.path.join(workdir, "m_%d.so" % abs(hash(name)))
    oracle.build_variant(src.replace(old, new), path)
    caught = []
    with oracle.using(path):
        for pin in pins:
            try:
                PINS[pin]()
            except AssertionError:
                caught.append(pin)
    assert caught, "no pin caught the mutant %r" % name
