"""Literal worked examples of the one-dimensional transforms.

Paper: arXiv 1903.07761, Sec. 2.3 ("Wavelet types") names the three schemes
(fourth-order interpolating W4, its lifted form W4_li, third-order
average-interpolating W3_ai) and the transform on the interval.  The values
below were derived by hand in exact rational arithmetic from the stencil
readings (W4: cubic through the four nearest evens at the odd position,
one-sided at the ends with cubic extrapolation for the last odd sample;
W4_li: W4 then the truncated centred update (-1, 9, 9, -1)/32 of the
details; W3_ai: pair averages, left child minus the average over its
half-cell of the quadratic matching three coarse averages).  Every value is
a short dyadic, so both precisions must reproduce them bit for bit, and the
inverse must return the input exactly.

Layout of each output: [coarse | details] after one level (n = 8), or
[coarse 4 | level-2 details 4 | level-1 details 8] after the full depth
(n = 16).
"""
import numpy as np
import pytest

DTYPES = [np.float32, np.float64]

QUARTIC = [0, 1, 16, 81, 256, 625, 1296, 2401]  # i^4
DIGITS = [3, 1, 4, 1, 5, 9, 2, 6]
CUBIC = [0, 1, 8, 27, 64, 125, 216, 343]  # i^3
SQUARE = [0, 1, 4, 9, 16, 25, 36, 49]  # i^2
DIGITS16 = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5, 8, 9, 7, 9, 3]

ONE_LEVEL_N8 = {
    "W4": {
        "quartic": [0, 16, 256, 1296, -15, 9, -15, 105],
        "digits": [3, 4, 5, 2, -2.25, -3.75, 4.75, 8.25],
        "cubic": [0, 8, 64, 216, 0, 0, 0, 0],
        "square": [0, 4, 16, 36, 0, 0, 0, 0],
    },
    "W4_li": {
        # coarse = evens + (-1, 9, 9, -1)/32 over the existing details
        "quartic": [-4.5, 473 / 32, 251.5, 42273 / 32, -15, 9, -15, 105],
        "digits": [159 / 64, 277 / 128, 163 / 32, 739 / 128, -2.25, -3.75, 4.75, 8.25],
        "cubic": [0, 8, 64, 216, 0, 0, 0, 0],
        "square": [0, 4, 16, 36, 0, 0, 0, 0],
    },
    "W3_ai": {
        "quartic": [0.5, 48.5, 440.5, 1848.5, -31.5, 22.5, 40.5, -73.5],
        "digits": [2, 2.5, 7, 4, 0.625, 2.125, -1.8125, -3.6875],
        "cubic": [0.5, 17.5, 94.5, 279.5, -3.75, 2.25, 2.25, -3.75],
        "square": [0.5, 6.5, 20.5, 42.5, 0, 0, 0, 0],
    },
}
INPUTS = {"quartic": QUARTIC, "digits": DIGITS, "cubic": CUBIC, "square": SQUARE}

FULL_N16 = {
    "W4": [3, 5, 5, 9, -0.625, -2.875, -1.125, -5.375,
           -2.25, -3.75, 5.625, 2.6875, -1.9375, 1, -3, -2],
    "W4_li": [1.7246856689453125, 4.564933776855469, 4.8037109375, 6.408546447753906,
              -2.780029296875, -0.710205078125, -1.052490234375, -6.677978515625,
              -2.25, -3.75, 5.625, 2.6875, -1.9375, 1, -3, -2],
    "W3_ai": [2.25, 5.5, 5.25, 7, 1, 1.875, -1.0625, 1.6875,
              0.625, 2.125, -1.8125, -2.375, 1.3125, -1, 0.9375, 2.0625],
}
# the coarse half after the first level only
LEVEL1_COARSE_N16 = {
    "W4": [3, 4, 5, 2, 5, 5, 9, 9],
    "W4_li": [2.484375, 2.13671875, 5.513671875, 4.515625, 5.00390625, 4.74609375, 8.560546875, 7.5625],
    "W3_ai": [2, 2.5, 7, 4, 4, 6.5, 8, 6],
}


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("scheme", ["W4", "W4_li", "W3_ai"])
@pytest.mark.parametrize("name", ["quartic", "digits", "cubic", "square"])
def test_one_level_n8_literal(oracle, scheme, name, dt):
    v = np.array(INPUTS[name], dt)
    want = np.array(ONE_LEVEL_N8[scheme][name], dt)
    got = oracle.fwd1(scheme, v)
    assert got.tobytes() == want.tobytes(), (scheme, name, got.tolist())
    back = oracle.inv1(scheme, want)
    assert back.tobytes() == v.tobytes(), (scheme, name, back.tolist())


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("scheme", ["W4", "W4_li", "W3_ai"])
def test_full_depth_n16_literal(oracle, scheme, dt):
    v = np.array(DIGITS16, dt)
    want = np.array(FULL_N16[scheme], dt)
    got = oracle.fwd_line(scheme, v)
    assert got.tobytes() == want.tobytes(), (scheme, got.tolist())
    assert oracle.fwd1(scheme, v)[:8].tobytes() == np.array(LEVEL1_COARSE_N16[scheme], dt).tobytes()
    assert oracle.inv_line(scheme, want).tobytes() == v.tobytes()


def test_cubic_and_quadratic_annihilation_literal():
    """The literal tables themselves: W4 and W4_li annihilate the cubic and the
    square; W3_ai annihilates only the square (its cubic details are the
    closed form (-15, 9, 9, -15)/4)."""
    for s in ("W4", "W4_li"):
        assert ONE_LEVEL_N8[s]["cubic"][4:] == [0, 0, 0, 0]
        assert ONE_LEVEL_N8[s]["square"][4:] == [0, 0, 0, 0]
    assert ONE_LEVEL_N8["W3_ai"]["square"][4:] == [0, 0, 0, 0]
    assert ONE_LEVEL_N8["W3_ai"]["cubic"][4:] == [-15 / 4, 9 / 4, 9 / 4, -15 / 4]
    # W4 and W4_li share their details (the update changes only the coarse half)
    for name in INPUTS:
        assert ONE_LEVEL_N8["W4"][name][4:] == ONE_LEVEL_N8["W4_li"][name][4:]
    assert FULL_N16["W4"][8:] == FULL_N16["W4_li"][8:]
