"""The float64 dense-SIFT oracle against its pins (tests/dsift_pins.py), and planted mistakes:
each mutated copy of the oracle must fail at least one pin."""
import types

import pytest

import dsift_pins as pins
import oracle.dsift as ds


@pytest.mark.parametrize("pin", pins.PINS, ids=[p.__name__ for p in pins.PINS])
def test_pin_holds(pin):
    pin(ds)


MUTATIONS = [
    ("central difference without the 1/2", "gx[:, 1:W - 1] = 0.5 * (", "gx[:, 1:W - 1] = 1.0 * ("),
    ("orientation not interpolated", "    f = t - b\n", "    f = 0.0 * (t - b)\n"),
    ("atan2 arguments swapped", "np.arctan2(gy, gx)", "np.arctan2(gx, gy)"),
    ("box instead of triangle", "return (B - abs(d)) / float(B * B)", "return 1.0 / float(2 * B - 1)"),
    ("x-major spatial bins", ".transpose(1, 2, 0)", ".transpose(2, 1, 0)"),
    ("no clamp", "v = np.minimum(v, CLAMP)", "v = v"),
    ("centre at the first bin", "(x0 + 1.5 * B + 0.5) / W", "(x0 + 0.5) / W"),
    ("resize without the half-pixel shift", "(np.arange(Ws) + 0.5) / s - 0.5", "np.arange(Ws) / s"),
    ("bin step not B", "F[:, y0:y0 + NBP * B:B, x0:x0 + NBP * B:B]",
     "F[:, y0:y0 + NBP * S:S, x0:x0 + NBP * S:S]"),
    ("one-sided difference reversed", "gx[:, 0] = img[:, 1] - img[:, 0]", "gx[:, 0] = img[:, 0] - img[:, 1]"),
]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(what, old, new):
    src = open(ds.__file__).read()
    assert src.count(old) == 1, what
    mod = types.ModuleType("dsift_mutant")
    exec(compile(src.replace(old, new), "dsift_mutant", "exec"), mod.__dict__)
    failed = []
    for pin in pins.PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError, KeyError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught: {what}"
