"""The Table 5.1 fixture is transcribed consistently: every printed rate is
the base-(n2/n1) logarithm of the printed error ratio (to the 4 decimals the
paper prints), and the errors fall with the printed orders."""
import math

from golden.table51 import RESOLUTIONS, load


def test_printed_rates_follow_from_printed_errors():
    errors, rates = load()
    assert len(errors) == 15 and len(rates) == 15
    checked = 0
    for key, r in rates.items():
        e = errors[key]
        order = int(key[0][3:])
        assert r[RESOLUTIONS[0]] is None
        for a, b in zip(RESOLUTIONS, RESOLUTIONS[1:]):
            if r[b] is None:
                assert e[b] is None
                continue
            rate = math.log(e[a] / e[b]) / math.log(b / a)
            assert abs(rate - r[b]) < 2e-3, (key, a, b, rate, r[b])
            assert abs(r[b] - order) < 0.2, (key, b, r[b])
            checked += 1
    assert checked == 54
