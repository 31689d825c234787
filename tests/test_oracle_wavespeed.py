"""Pin of the oracle's HLLC wave-speed estimate against the exact Riemann solver.

The wave speeds of eq. hllc-mixed-dvel are s_L = u_L - c_L q_L and
s_R = u_R + c_R q_R with q_K = sqrt(1 + (gamma+1)/(2 gamma) (p*/p_K - 1)) when
p* > p_K, and p* is the primitive-variable (linearised) pressure estimate.
The exact solution gives two independent facts to check this against:

* For weak waves the linearised Riemann problem is exact to first order: with
  jumps of size eps, the exact star pressure differs from the linearised one
  by O(eps^2).
* With the exact p*, the q formula is the exact Rankine-Hugoniot shock speed,
  so with the estimate it is off by O(eps^2) as well.  The exact shock speed
  is taken here from mass conservation across the sampled shock,
  (rho* u* - rho_K u_K) / (rho* - rho_K), which uses the Hugoniot density ratio
  and not the q formula.

A wrong coefficient in the pressure estimate or in q_K leaves an O(eps) error,
which the measured order of convergence exposes.  The second test plants such
mistakes in a copy of the oracle source and checks that the pin catches each.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from oracle import build as OB

EPS = (4e-3, 2e-3, 1e-3)


def _cases(n=12):
    """Seeded weak two-shock problems: a base state and perturbation
    directions with u_L > u_R, so both waves are shocks (p* > p_L, p_R)."""
    rng = np.random.default_rng(4242)
    out = []
    for i in range(n):
        g = (1.4, 5.0 / 3.0)[i % 2]
        rho0 = float(np.exp(rng.uniform(-1, 1)))
        p0 = float(np.exp(rng.uniform(-1, 1)))
        u0 = float(rng.uniform(-1, 1))
        a = rng.uniform(-0.25, 0.25, 4)  # relative density / pressure directions
        b = rng.uniform(0.5, 1.5, 2)     # closing velocities, in units of c0
        out.append((g, rho0, u0, p0, a, b))
    return out


def _states(case, eps):
    g, rho0, u0, p0, a, b = case
    c0 = np.sqrt(g * p0 / rho0)
    WL = np.array([rho0 * (1 + eps * a[0]), u0 + eps * c0 * b[0], p0 * (1 + eps * a[1])])
    WR = np.array([rho0 * (1 + eps * a[2]), u0 - eps * c0 * b[1], p0 * (1 + eps * a[3])])
    return g, WL, WR


def _exact_shock_speeds(g, WL, WR):
    """p* and the two shock speeds of the exact solution, the speeds from
    mass conservation across the sampled star states."""
    ps, us = O.exact_star(g, WL, WR, method=1)
    assert ps > WL[2] and ps > WR[2], "both waves must be shocks"
    rl_star = O.exact_sample(g, WL, WR, [us - 1e-7])[0, 0]
    rr_star = O.exact_sample(g, WL, WR, [us + 1e-7])[0, 0]
    SL = (rl_star * us - WL[0] * WL[1]) / (rl_star - WL[0])
    SR = (rr_star * us - WR[0] * WR[1]) / (rr_star - WR[0])
    return ps, SL, SR


def _hllc_speeds(hllc_detail, g, WL, WR):
    d = hllc_detail(g, WL, WR)
    return d["p_star"], d["sL"], d["sR"]


def _orders(hllc_detail):
    """Observed orders log2(e(eps)/e(eps/2)) of the p*, s_L and s_R errors
    over the cases, per quantity (rows) and refinement (columns)."""
    orders = []
    for case in _cases():
        errs = []
        for eps in EPS:
            g, WL, WR = _states(case, eps)
            ex = _exact_shock_speeds(g, WL, WR)
            est = _hllc_speeds(hllc_detail, g, WL, WR)
            errs.append([abs(e - x) for e, x in zip(est, ex)])
        errs = np.array(errs)  # [eps][quantity]
        orders.append(np.log2(errs[:-1] / errs[1:]).T)
    return np.array(orders)  # [case][quantity][refinement]


def _oracle_detail(g, WL, WR):
    return O.hllc(g, WL, WR, detail=True)[1]


def test_wave_speed_estimate_second_order_in_weak_waves():
    """p*, s_L and s_R of the oracle approach the exact two-shock solution
    as eps^2 (order 2 +- 0.25 at every refinement of every case)."""
    orders = _orders(_oracle_detail)
    assert orders.shape == (12, 3, 2)
    assert np.all(np.abs(orders - 2.0) < 0.25), orders


def test_wave_speed_error_level_is_quadratic():
    """Absolute level: error / eps^2 stays bounded (a few units of the base
    state's scales) as eps shrinks, for p* / p0 and s_K / c0."""
    for case in _cases():
        g, rho0, u0, p0, a, b = case
        c0 = np.sqrt(g * p0 / rho0)
        for eps in EPS:
            g, WL, WR = _states(case, eps)
            ps, SL, SR = _exact_shock_speeds(g, WL, WR)
            d = _oracle_detail(g, WL, WR)
            assert abs(d["p_star"] - ps) / p0 <= 5.0 * eps ** 2
            assert abs(d["sL"] - SL) / c0 <= 5.0 * eps ** 2
            assert abs(d["sR"] - SR) / c0 <= 5.0 * eps ** 2


# ------------------------------------------------------------------ mutants

MUTANTS = {
    "pressure-estimate coefficient 1/8 -> 1/4": ("0.125 * (ur - ul)", "0.25 * (ur - ul)"),
    "q factor (g+1)/(2g) -> (g-1)/(2g)": ("double z = (g + 1.0) / (2.0 * g);",
                                          "double z = (g - 1.0) / (2.0 * g);"),
    "mean pressure uses p_L twice": ("0.5 * (pl + pr) - 0.125", "0.5 * (pl + pl) - 0.125"),
    "sound-speed sum -> difference": ("(rl + rr) * (cl + cr)", "(rl + rr) * (cl - cr)"),
    "velocity jump reversed": ("0.125 * (ur - ul)", "0.125 * (ul - ur)"),
}


def _build_mutant(tmp_path, old, new):
    src = os.path.join(OB.HERE, "hydro_oracle.c")
    text = open(src).read()
    assert text.count(old) == 1, old
    d = tmp_path / "mut"
    d.mkdir()
    (d / "hydro_oracle.c").write_text(text.replace(old, new))
    shutil.copy(os.path.join(OB.HERE, "exact_riemann.c"), d / "exact_riemann.c")
    shutil.copy(os.path.join(OB.HERE, "hydro_oracle.h"), d / "hydro_oracle.h")
    so = d / "libmut.so"
    cmd = ["gcc", *OB.FLAGS, "-o", str(so), str(d / "hydro_oracle.c"), str(d / "exact_riemann.c"), "-lm"]
    subprocess.run(cmd, check=True)
    L = C.CDLL(str(so))
    dp = C.POINTER(C.c_double)
    L.orc_hllc.restype = None
    L.orc_hllc.argtypes = [C.c_double, C.c_int, dp, dp, dp, dp]

    def detail(g, WL, WR):
        WL = np.ascontiguousarray(WL, dtype=np.float64)
        WR = np.ascontiguousarray(WR, dtype=np.float64)
        F = np.empty(3)
        det = np.empty(4 + 8 * 3)
        L.orc_hllc(float(g), 0, WL.ctypes.data_as(dp), WR.ctypes.data_as(dp), F.ctypes.data_as(dp),
                   det.ctypes.data_as(dp))
        return {"sL": det[0], "s_star": det[1], "sR": det[2], "p_star": det[3]}

    return detail


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pin_catches_planted_mistake(tmp_path, name):
    """A mistake planted in a copy of the oracle's wave-speed code (the
    committed oracle is untouched) drops the observed order below 1.5."""
    old, new = MUTANTS[name]
    detail = _build_mutant(tmp_path, old, new)
    orders = _orders(detail)
    assert not np.all(np.abs(orders - 2.0) < 0.25), name
    assert np.median(orders) < 1.5, (name, np.median(orders))
