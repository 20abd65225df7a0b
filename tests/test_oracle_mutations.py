"""Plant one mistake at a time in the oracle (on the CPU) and check that the
pins catch it: each planted build must fail at least one pin.

The mistakes are compiled into ``oracle.c`` behind ``ORACLE_MUTATION`` (off
in the real build): a sign, an index, a wrap-around, a normalisation, a
scale, a dropped term, a dropped axis, a crop offset, a twiddle exponent and
a wrong power law.
"""
import numpy as np
import pytest

import oracle
import test_oracle_box as box
import test_oracle_pins as pins

MUTATIONS = {
    1: "self-cell value with the wrong sign",
    2: "kernel wrap-around off by one",
    3: "conjugated radix-2 twiddles",
    4: "inverse transform not divided by P^3",
    5: "dx^2 instead of dx^3",
    6: "direct sum drops the self term",
    7: "3D transform skips the z axis",
    8: "crop shifted by one cell in x",
    9: "combine twiddle exponent uses k instead of k + s m",
    10: "1/r^2 kernel instead of 1/r",
    11: "box self cell ignores the spacings",
    12: "y and z spacings swapped in the kernel on dx x dy x dz cells",
    13: "dx^3 instead of dx dy dz as the cell volume",
    14: "box convolution normalised by Px Px Pz instead of Px Py Pz",
    15: "y and z displacements exchanged in the padded box kernel",
}

CHECKS = [
    lambda o: pins.test_fft_matches_bruteforce_dft(o, 12),
    lambda o: pins.test_fft_matches_numpy(o, 96),
    lambda o: pins.test_fft3_matches_numpy_axes(o, 6),
    lambda o: pins.test_fft_conv_equals_direct_sum_small(o, 8, 1),
    lambda o: pins.test_single_cell_worked_example(o),
    lambda o: pins.test_impulse_response_is_the_kernel(o, 12, (0, 11, 6)),
    lambda o: pins.test_green_hat_real_and_even(o, 6),
    lambda o: pins.test_gaussian_sphere_closed_form_second_order(o),
    lambda o: pins.test_box_self_cell_scales_like_the_cube(o),
    lambda o: pins.test_anisotropic_impulse_response_and_axis_swap(o),
    lambda o: pins.test_anisotropic_monopole_far_field(o),
    lambda o: box.test_box_fft_conv_equals_direct_sum(o, (6, 10, 8), (0.1, 0.13, 0.07)),
    lambda o: box.test_box_kernel_pad_is_even_per_axis(o),
]


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("planted")
    return {m: oracle.variant(oracle.build_variant(str(d / f"liboracle_m{m}.so"), [f"ORACLE_MUTATION={m}"]))
            for m in MUTATIONS}


def _failures(o):
    failed = []
    for k, check in enumerate(CHECKS):
        try:
            check(o)
        except (AssertionError, RuntimeError, ValueError, FloatingPointError):
            failed.append(k)
    return failed


def test_unmutated_build_passes_every_check(tmp_path):
    o = oracle.variant(oracle.build_variant(str(tmp_path / "liboracle_m0.so"), ["ORACLE_MUTATION=0"]))
    assert _failures(o) == []


@pytest.mark.parametrize("m", sorted(MUTATIONS))
def test_planted_mistake_is_caught(builds, m):
    with np.errstate(all="ignore"):
        failed = _failures(builds[m])
    print(f"mutation {m} ({MUTATIONS[m]}): caught by checks {failed}")
    assert failed, f"no pin catches: {MUTATIONS[m]}"
