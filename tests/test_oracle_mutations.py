"""Plausible mistakes planted in a copy of the oracle must fail its pins.

Each mutation rewrites one expression of ``oracle/oracle.c`` in a temporary
copy (the separable Smith product instead of the height-correlated form, a
wrong Schlick power or argument, the step factor dropped from the SVGF depth
weight, ...), builds it with the oracle's own flags and runs the pins against
it: at least one pin has to fail, so that the pins, not just the oracle's
agreement with the GPU, fix what the oracle computes.  CPU only.
"""
import concurrent.futures as cf
import ctypes as C
import os
import subprocess

import pytest

from oracle import oracle as O

import test_oracle_pins_terms as T

MUTATIONS = {
    # specular lobe
    "separable_smith": ("t->Vis = 0.5 / (t->A + t->B);",
                        "t->Vis = 1.0 / ((NdotV + t->sv) * (t->NdotL + t->sl));"),
    "schlick_power_4": ("t->P = pow(1.0 - t->VdotH, 5.0);", "t->P = pow(1.0 - t->VdotH, 4.0);"),
    "schlick_of_n_dot_h": ("t->P = pow(1.0 - t->VdotH, 5.0);", "t->P = pow(1.0 - t->NdotH, 5.0);"),
    "ggx_denominator_not_squared": ("t->D = t->a2 / (M_PI * t->Q * t->Q);",
                                    "t->D = t->a2 / (M_PI * t->Q);"),
    "alpha_is_roughness": ("double alpha = r * r;\n    t->a2", "double alpha = r;\n    t->a2"),
    # denoiser
    "depth_step_dropped": ("fabs(gx[p] * i * step + gy[p] * j * step)", "fabs(gx[p] * i + gy[p] * j)"),
    "depth_axes_swapped": ("fabs(gx[p] * i * step + gy[p] * j * step)",
                           "fabs(gy[p] * i * step + gx[p] * j * step)"),
    "variance_window_5x5": ("for (int dy = -3; dy <= 3; ++dy)\n                for (int dx = -3; dx <= 3; ++dx)",
                            "for (int dy = -2; dy <= 2; ++dy)\n                for (int dx = -2; dx <= 2; ++dx)"),
    "variance_weights_not_squared": ("vacc += w * w * var[q];", "vacc += w * var[q];"),
    "luminance_weight_without_sqrt": ("sl * sqrt(g3[p] > 0 ? g3[p] : 0)", "sl * (g3[p] > 0 ? g3[p] : 0)"),
    "variance_blur_dropped": ("sl * sqrt(g3[p] > 0 ? g3[p] : 0)", "sl * sqrt(var[p] > 0 ? var[p] : 0)"),
}


def _build(name, src, tmpdir):
    pat, rep = MUTATIONS[name]
    assert src.count(pat) == 1, f"mutation {name}: pattern not found once in oracle.c"
    c_path = os.path.join(tmpdir, f"or_{name}.c")
    so_path = os.path.join(tmpdir, f"libor_{name}.so")
    with open(c_path, "w") as f:
        f.write(src.replace(pat, rep))
    subprocess.check_call(["gcc", *O.GCC_FLAGS, "-o", so_path, c_path, "-lm"])
    return name, so_path


@pytest.fixture(scope="module")
def mutated_libs(tmp_path_factory):
    tmpdir = str(tmp_path_factory.mktemp("oracle_mutants"))
    with open(O._SRC) as f:
        src = f.read()
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(lambda n: _build(n, src, tmpdir), MUTATIONS))


def _failing_pins(lib_path):
    h = C.CDLL(lib_path)
    O._set_types(h)
    saved = O._lib
    O._lib = h
    failed = []
    try:
        for pin in T.PINS:
            try:
                pin()
            except AssertionError:
                failed.append(pin.__name__)
    finally:
        O._lib = saved
    return failed


def test_unmutated_oracle_passes_every_pin():
    assert _failing_pins(O.build(force=False)) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name, mutated_libs):
    failed = _failing_pins(mutated_libs[name])
    assert failed, f"mutation {name} passes every pin"
