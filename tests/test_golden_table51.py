"""The Table 5.1 fixture is transcribed consistently: every printed rate is
the base-(n2/n1) logarithm of the printed error ratio (to the 4 decimals the
paper prints)."""
import math

from golden.table51 import RESOLUTIONS, load


def test_printed_rates_follow_from_printed_errors():
    errors, rates = load()
    assert len(errors) == 4 and len(rates) == 4
    for key, r in rates.items():
        e = errors[key]
        for (a, b), printed in zip(zip(RESOLUTIONS, RESOLUTIONS[1:]), r):
            rate = math.log(e[a] / e[b]) / math.log(b / a)
            assert abs(rate - printed) < 2e-3, (key, a, b, rate, printed)
