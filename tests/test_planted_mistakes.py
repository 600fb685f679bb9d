"""The oracle's pins catch plausible mistakes.  Each case compiles the oracle
with one deliberate mistake (a wrong sign, a dropped term, a transposed
operand, a wrong index, a wrong rounding) into its own library, swaps it in
for the oracle's own, and checks that the named pins fail on it while they
pass on the real oracle.  The blob layout's mistake is planted in Python,
around the oracle's own elision routine.  CPU only."""
import numpy as np
import pytest

import oracle as O
import tests.test_oracle_pins as P

# plant number (SZO_PLANT in the oracle's C source) -> pins that must catch it
CASES = {
    1: ("NAK outer taps with the wrong sign (Sec. V-B.1)",
        [P.test_spline_exactness_on_polynomials, P.test_spline_weights_match_lagrange_and_paper]),
    2: ("natural cubic with its outer term dropped (Sec. V-B.1)",
        [P.test_spline_exactness_on_polynomials, P.test_spline_weights_match_lagrange_and_paper]),
    3: ("left quadratic reading x[n+3] for x[n-3] (Sec. V-B.1)",
        [P.test_spline_exactness_on_polynomials, P.test_spline_weights_match_lagrange_and_paper]),
    4: ("quantiser truncating instead of rounding (Sec. III-A)",
        [lambda: P.test_quantiser_round_half_even_and_radius(1.5, 514),
         lambda: P.test_quantiser_round_half_even_and_radius(3.5, 516)]),
    5: ("error bound rounded to nearest instead of down",
        [P.test_round_down_is_largest_float_below]),
    6: ("level bounds shifted by one level (Sec. V-B.2)",
        [P.test_level_bounds_exact_rational]),
    7: ("canonical codes counting the wrong length (Sec. VI-A)",
        [P.test_canonical_codes_rfc1951_example]),
    8: ("profiling keeping the cubic with the larger error (Sec. V-C.1)",
        [P.test_profile_cubic_along_x_picks_nak, P.test_profile_cosine_picks_natural]),
    9: ("smoothest dimension first (Sec. V-C.2)",
        [P.test_profile_order_least_smooth_first]),
    10: ("x[n+3] unavailable at the window's last point (Sec. V-B.1, V-D)",
         [P.test_spline_map_matches_paper_figure]),
    11: ("each code's bits written least significant first (Sec. VI-A)",
         [P.test_bitstream_hand_example]),
    12: ("Eq. 1 falling instead of rising between 1e-3 and 1e-2",
         [P.test_alpha_piecewise_linear_and_continuous]),
    13: ("relative bound scaled by the maximum instead of the range (Sec. V-C.1)",
         [P.test_level_bounds_exact_rational]),
}


def setup_module(module):
    O.build(force=False)


@pytest.mark.parametrize("plant", sorted(CASES), ids=[CASES[k][0] for k in sorted(CASES)])
def test_pins_catch_planted_mistake(plant, tmp_path, monkeypatch):
    what, pins = CASES[plant]
    for pin in pins:          # the real oracle passes them
        pin()
    path = O.build(plant=plant, out=str(tmp_path / ("libszo_plant%d.so" % plant)))
    monkeypatch.setattr(O, "_lib", O.load(path))
    for pin in pins:
        with pytest.raises(AssertionError):
            pin()


_real_elide = O.elide_zero_words


def _bitmap_msb_first(words):
    """The oracle's elision with the bitmap's bit order reversed (word k
    marked by bit 31 - k % 32): a planted mistake in the blob layout."""
    e = _real_elide(words)
    if e is None:
        return None
    nbm = (np.asarray(words).size + 31) // 32
    bm = e[:nbm].copy()
    rev = np.zeros_like(bm)
    for b in range(32):
        rev |= ((bm >> np.uint32(b)) & np.uint32(1)) << np.uint32(31 - b)
    e[:nbm] = rev
    return e


def test_pins_catch_planted_bitmap_order(monkeypatch):
    P.test_zero_word_elision_layout()
    monkeypatch.setattr(O, "elide_zero_words", _bitmap_msb_first)
    with pytest.raises(AssertionError):
        P.test_zero_word_elision_layout()
