"""Each plausible mistake planted in the oracle (on the CPU) makes at least
one pin fail, and the pins pass again once it is removed.

Planted mistakes: 1 pull-back with J^-1 in place of J^-T (the transpose
question of Example 1), 2 a dropped quadrature weight, 3 a dropped |det J|,
4 a sign slip in the inverse, 5 the coefficient evaluated away from the
physical point G(xhat), 6 the convection derivative on the test function
instead of the trial function (full assembly only).
"""
import numpy as np
import pytest

import oracle
from tests import test_oracle_conv as conv_pins
from tests import test_oracle_pins as pins

PIN_CASES = [
    ("patch test 2D", lambda: pins.test_patch_test_2d((4, 5), 2)),
    ("affine map 2D", lambda: pins.test_affine_map_2d(np.array([[1.0, 0.3], [0.2, 1.1]]))),
    ("domain area 2D", lambda: pins.test_mass_sum_equals_domain_area_2d((4, 5), 2)),
    ("dense brute force 2D", lambda: pins.test_dense_bruteforce_algebraic_form(2, (3, 4), 2, ("sinprod", 0.5))),
    ("dense brute force 3D", lambda: pins.test_dense_bruteforce_algebraic_form(3, (2, 3, 2), 3, ("sinprod", 0.5))),
    ("identity Kronecker", lambda: pins.test_identity_geometry_is_kronecker(2, (5, 4), 3)),
    ("linear functions, evaluation", lambda: pins.test_eval_reproduces_linear_physical_functions(3, (3, 2, 4), 2)),
]

# the convection form's pins, with the plants that touch it
CONV_PIN_CASES = [
    ("convection 1D by parts", lambda: conv_pins.test_1d_integration_by_parts(7, 3)),
    ("convection identity Kronecker", lambda: conv_pins.test_identity_map_is_kronecker((3, 2, 3), 3)),
    ("convection affine map 2D", lambda: conv_pins.test_affine_map_2d(np.array([[1.0, 0.3], [0.2, 1.1]]))),
    ("convection coordinate function",
     lambda: conv_pins.test_coordinate_function_on_curved_maps(3, (3, 2, 3), 2, ("const", 0.8))),
]


def _failing_pins(cases=PIN_CASES):
    failed = []
    for name, case in cases:
        try:
            case()
        except (AssertionError, oracle.OracleError):
            failed.append(name)
    return failed


@pytest.fixture
def planted():
    yield oracle.set_defect
    oracle.set_defect(0)


@pytest.mark.parametrize("defect", [1, 2, 3, 4, 5])
def test_planted_mistake_is_caught(planted, defect):
    planted(defect)
    failed = _failing_pins()
    planted(0)
    assert failed, f"planted mistake {defect} passed every pin"


def test_pins_pass_without_plant(planted):
    planted(0)
    assert _failing_pins() == []


@pytest.mark.parametrize("defect", [1, 2, 3, 4, 6])
def test_planted_mistake_is_caught_by_the_convection_pins(planted, defect):
    planted(defect)
    failed = _failing_pins(CONV_PIN_CASES)
    planted(0)
    assert failed, f"planted mistake {defect} passed every convection pin"


def test_convection_pins_pass_without_plant(planted):
    planted(0)
    assert _failing_pins(CONV_PIN_CASES) == []
