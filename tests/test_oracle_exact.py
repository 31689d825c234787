"""Pins of the exact Riemann solver that validates the oracle scheme.

Checked against gas dynamics written independently of the solver's own
formulas: the conservation form of the Rankine-Hugoniot conditions across
the sampled shocks, the Riemann invariant and entropy across fans, the
closed-form star pressure of two rarefactions, and symmetry.
"""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl


def cons(rho, u, p, g):
    return np.array([rho, rho * u, p / (g - 1) + 0.5 * rho * u * u])


def flux(rho, u, p, g):
    E = p / (g - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, (E + p) * u])


@pytest.mark.parametrize("seed", range(102, 122))
def test_newton_and_bisection_agree(seed):
    left, right = wl.random_two_state(seed)
    p1, u1 = O.exact_star(1.4, left, right, method=0)
    p2, u2 = O.exact_star(1.4, left, right, method=1)
    assert abs(p1 - p2) <= 1e-13 * p1
    assert abs(u1 - u2) <= 1e-12 * (1 + abs(u1))


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_two_rarefaction_closed_form(g):
    """When both waves are rarefactions p* has a closed form."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        rl, rr, pl, pr = np.exp(rng.uniform(-1, 1, 4))
        cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
        du = rng.uniform(0.2, 0.9) * 2 * (cl + cr) / (g - 1)  # receding, no vacuum
        ul, ur = -0.5 * du, 0.5 * du
        z = (g - 1) / (2 * g)
        want = ((cl + cr - 0.5 * (g - 1) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1 / z)
        for method in (0, 1):
            ps, us = O.exact_star(g, (rl, ul, pl), (rr, ur, pr), method=method)
            assert ps <= min(pl, pr)
            assert abs(ps - want) <= 1e-11 * want


@pytest.mark.parametrize("seed", [103, 104, 105, 106, 107])
def test_rankine_hugoniot_conservation_across_shocks(seed):
    """Each pressure jump from the uniform outer states to the star states that
    is a shock satisfies s [U] = [F] with one speed s for all components."""
    g = 1.4
    left, right = wl.random_two_state(seed)
    ps, us = O.exact_star(g, left, right)
    rl, ul, pl = left
    rr, ur, pr = right
    if ps > pl:
        # left shock: star density from the sampled solution just left of the contact
        r, u, p = O.exact_sample(g, left, right, [us - 1e-9])[:, 0]
        U1, U2 = cons(rl, ul, pl, g), cons(r, u, p, g)
        F1, F2 = flux(rl, ul, pl, g), flux(r, u, p, g)
        s = (F2[0] - F1[0]) / (U2[0] - U1[0])
        assert np.allclose(s * (U2 - U1), F2 - F1, rtol=1e-10, atol=1e-12)
        assert s < ul  # moves left relative to the fluid
    if ps > pr:
        r, u, p = O.exact_sample(g, left, right, [us + 1e-9])[:, 0]
        U1, U2 = cons(rr, ur, pr, g), cons(r, u, p, g)
        F1, F2 = flux(rr, ur, pr, g), flux(r, u, p, g)
        s = (F2[0] - F1[0]) / (U2[0] - U1[0])
        assert np.allclose(s * (U2 - U1), F2 - F1, rtol=1e-10, atol=1e-12)
        assert s > ur


@pytest.mark.parametrize("seed", [108, 109, 110, 111])
def test_rarefaction_invariants(seed):
    """Across a left (right) fan, u + 2c/(g-1) (u - 2c/(g-1)) and p/rho^g are constant."""
    g = 1.4
    left, right = wl.random_two_state(seed)
    ps, us = O.exact_star(g, left, right)
    for side, state, sign in ((0, left, 1.0), (1, right, -1.0)):
        rk, uk, pk = state
        if ps > pk:
            continue
        ck = np.sqrt(g * pk / rk)
        head = uk - sign * ck
        eps = 1e-9 * (1 + abs(us))
        if side == 0:
            xi = np.linspace(head - 0.5, us - eps, 400)
        else:
            xi = np.linspace(us + eps, head + 0.5, 400)
        r, u, p = O.exact_sample(g, left, right, xi)
        c = np.sqrt(g * p / r)
        inv = u + sign * 2 * c / (g - 1)
        assert np.allclose(inv, uk + sign * 2 * ck / (g - 1), rtol=1e-12, atol=1e-12)
        assert np.allclose(p / r ** g, pk / rk ** g, rtol=1e-11)


def test_symmetric_collision_and_expansion():
    for u in (0.5, -0.5, 2.0):
        ps, us = O.exact_star(1.4, (1.0, u, 1.0), (1.0, -u, 1.0))
        assert abs(us) <= 1e-14
        if u > 0:
            assert ps > 1.0
        else:
            assert ps < 1.0


def test_contact_continuity():
    left, right = wl.random_two_state(112)
    ps, us = O.exact_star(1.4, left, right)
    a = O.exact_sample(1.4, left, right, [us - 1e-12, us + 1e-12])
    assert np.allclose(a[1], us, rtol=1e-12) and np.allclose(a[2], ps, rtol=1e-12)


def test_vacuum_rejected():
    with pytest.raises(O.OracleError):
        O.exact_star(1.4, (1.0, -10.0, 1.0), (1.0, 10.0, 1.0))
