"""Pins of the reference solutions in tests/refsol.py (which in turn pin the
oracle) against values printed in the literature (tests/golden/*.txt, each
file naming its source)."""
import os

import pytest

from refsol import ExactRiemann, sedov_xi0

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def _close(got, want_text):
    """Agreement to the printed figures: within a unit of the last printed
    digit (the book truncates some entries rather than rounding them), or
    1e-5 relative for the six-figure entries."""
    want = float(want_text)
    digits = want_text.split(".")[1] if "." in want_text else ""
    ulp = 10.0 ** (-len(digits))
    return abs(got - want) <= max(ulp, 1e-5 * abs(want))


@pytest.mark.parametrize("row", list(_rows("toro_exact_riemann_star.txt")))
def test_exact_riemann_star_states(row):
    left, right = row.split("|")
    f = left.split()
    test = int(f[0])
    rl, ul, pl, rr, ur, pr = map(float, f[1:])
    want = right.split()
    s = ExactRiemann(rl, ul, pl, rr, ur, pr, 1.4)
    got = [s.pstar, s.ustar, s.rstar_l, s.rstar_r]
    for g, w, name in zip(got, want, ["p*", "u*", "rho*L", "rho*R"]):
        assert _close(g, w), (test, name, g, w)


def test_sedov_constant():
    for row in _rows("sedov_alpha.txt"):
        gam, alpha = map(float, row.split())
        xi0 = sedov_xi0(gam)
        assert abs(xi0 ** -5 - alpha) <= 6e-4, (gam, xi0 ** -5, alpha)
