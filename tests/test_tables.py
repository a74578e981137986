"""Pins for the constant tables the HIP kernels compile in (csrc/tables.h), read from the
header text and checked without the generator: the quadrature rules integrate every
monomial of degree <= 4 exactly on the reference simplex, and the star mass moments
add up to int phi_0 = 1 (unit lattice)."""
import itertools
import math
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1502_04657_amd", "csrc",
                   "tables.h")


def _array(name):
    text = open(HDR).read()
    m = re.search(r"%s\[[^=]*=\s*\{(.*?)\};" % re.escape(name), text, flags=re.S)
    assert m, name
    return np.array([float(v) for v in re.findall(r"-?\d+(?:\.\d+)?(?:[eE][-+]?\d+)?", m.group(1))])


def _exact(mon):
    # int over the unit simplex of prod l_i^a_i / volume = d! prod a_i! / (d + sum a)!
    d = len(mon) - 1
    num = math.factorial(d)
    for a in mon:
        num *= math.factorial(a)
    return num / math.factorial(d + sum(mon))


def _check_rule(pts, wts, nb):
    pts = pts.reshape(-1, nb)
    assert len(pts) == len(wts)
    assert np.allclose(pts.sum(axis=1), 1.0, atol=1e-15)
    for mon in itertools.product(range(5), repeat=nb):
        if sum(mon) > 4:
            continue
        q = float(np.sum(wts * np.prod(pts ** np.array(mon), axis=1)))
        assert abs(q - _exact(mon)) <= 2e-16 * max(1.0, abs(_exact(mon))) * 8, (mon, q, _exact(mon))


def test_triangle_rule_is_exact_to_degree_4():
    _check_rule(_array("kQuadPt2D"), _array("kQuadW2D"), 3)


def test_tetrahedron_rule_is_exact_to_degree_4():
    _check_rule(_array("kQuadPt3D"), _array("kQuadW3D"), 4)


def test_star_mass_moments_integrate_the_hat():
    for name in ("kM0_2D", "kM0_3D"):
        assert abs(_array(name).sum() - 1.0) < 1e-15
