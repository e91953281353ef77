"""Closed-form integrals used to pin the error norms (oracle and GPU): monomials over the
unit simplex in exact rational arithmetic, and the three error sums of u = x^2 y^2 z^2
against u_h = 0, lambda = 0 on the unit tet."""
from fractions import Fraction
from math import factorial, sqrt


def simplex_monomial(e, dim):
    """integral of prod x_i^e_i over the unit dim-simplex (the last coordinate 1 - sum of the
    others when len(e) = dim + 1)"""
    num = 1
    for a in e:
        num *= factorial(a)
    return Fraction(num, factorial(sum(e) + dim))


def unit_tet_x2y2z2(h):
    """(grad2, l22, lam_h2) for u = x^2 y^2 z^2 on the unit tet, u_h = 0, lambda = 0, mesh
    size h: ||grad u||^2, ||u||^2 and h sum_F ||grad u . nu||^2_F."""
    # ||u||^2 = int x^4 y^4 z^4;  ||grad u||^2 = 3 * 4 int x^2 y^4 z^4
    l22 = simplex_monomial((4, 4, 4), 3)
    grad2 = 12 * simplex_monomial((2, 4, 4), 3)
    # faces x = 0, y = 0, z = 0: grad u . nu = 0; face x + y + z = 1: grad u . nu =
    # 2 xyz (xy + yz + zx) / sqrt 3, dS = sqrt 3 dx dy on the projected triangle
    sq = {}
    for a, b, w in [((1, 1, 0), (1, 1, 0), 1), ((0, 1, 1), (0, 1, 1), 1), ((1, 0, 1), (1, 0, 1), 1),
                    ((1, 1, 0), (0, 1, 1), 2), ((1, 1, 0), (1, 0, 1), 2), ((0, 1, 1), (1, 0, 1), 2)]:
        m = tuple(2 + i + j for i, j in zip(a, b))  # x^2 y^2 z^2 (xy + yz + zx)^2 term by term
        sq[m] = sq.get(m, 0) + w
    face = sum(w * simplex_monomial(m, 2) for m, w in sq.items())  # int over the projected triangle
    lam_h2 = h * 4 / 3 * sqrt(3) * float(face)
    return float(grad2), float(l22), lam_h2
