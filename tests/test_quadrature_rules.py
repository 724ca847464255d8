"""The quadrature rules behind the generated P2/P3 action (act_q): each must
integrate every monomial of its degree exactly on the reference simplex
(rational arithmetic, against the closed form a!/(|a|+d)!), and not every
monomial of the next degree (so the check has teeth)."""
import itertools
import os
import sys
from fractions import Fraction
from math import factorial

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", "paper_1501_01809_amd", "csrc"))
import gen_tables as G  # noqa: E402


def _exact(a, d):
    num = 1
    for x in a:
        num *= factorial(x)
    return Fraction(num, factorial(sum(a) + d))


def _max_exact_degree(d, rule, cap=8):
    for deg in range(cap + 1):
        for a in itertools.product(range(deg + 1), repeat=d + 1):
            if sum(a) != deg:
                continue
            q = sum(w * G.poly_eval({a: Fraction(1)}, pt) for w, pt in rule)
            if q != factorial(d) * _exact(a, d):
                return deg - 1
    return cap


@pytest.mark.parametrize("d,rule,degree", [
    (2, G.QRULES[2], 3), (3, G.QRULES[3], 3), (2, G.gm_rule(2, 2), 5), (3, G.gm_rule(3, 2), 5)])
def test_rule_degree(d, rule, degree):
    assert sum(w for w, _ in rule) == 1
    assert all(sum(pt) == 1 for _, pt in rule)
    assert _max_exact_degree(d, rule) == degree


def test_rule_sizes():
    assert len(G.QRULES[3]) == 5 and len(G.QRULES[2]) == 4
    assert len(G.gm_rule(3, 2)) == 15 and len(G.gm_rule(2, 2)) == 10
