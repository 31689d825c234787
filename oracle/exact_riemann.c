/*
 * exact_riemann.c -- TEST INFRASTRUCTURE ONLY (see hydro_oracle.h).
 *
 * Exact solution of the Riemann problem of the 1-D Euler equations for a
 * gamma-law gas (eq. hydro).  Used only to validate the oracle scheme against
 * shock-tube data (Sec. 4.2 compares the solver with semi-analytic solutions).
 *
 * Textbook gas dynamics: the star pressure solves f_L(p) + f_R(p) + (u_R - u_L)
 * = 0 where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the
 * isentropic rarefaction branch for p <= p_K; the star velocity is
 * (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  Two independent root finders are
 * provided (Newton, bisection) so each can check the other.
 */
#include <math.h>

#include "hydro_oracle.h"

static void pressure_fn(double g, double p, double rk, double pk, double ck, double* f,
                        double* df) {
    if (p <= pk) {
        /* rarefaction: f = 2c/(g-1) [ (p/pk)^((g-1)/(2g)) - 1 ] */
        double r = p / pk;
        *f = 2.0 * ck / (g - 1.0) * (pow(r, (g - 1.0) / (2.0 * g)) - 1.0);
        *df = pow(r, -(g + 1.0) / (2.0 * g)) / (rk * ck);
    } else {
        /* shock: f = (p - pk) sqrt(A / (p + B)), A = 2/((g+1) rk), B = pk (g-1)/(g+1) */
        double A = 2.0 / ((g + 1.0) * rk);
        double B = pk * (g - 1.0) / (g + 1.0);
        double s = sqrt(A / (p + B));
        *f = (p - pk) * s;
        *df = s * (1.0 - 0.5 * (p - pk) / (p + B));
    }
}

static double total_fn(double g, double p, double rl, double ul, double pl, double cl, double rr,
                       double ur, double pr, double cr, double* df) {
    double fl, dfl, fr, dfr;
    pressure_fn(g, p, rl, pl, cl, &fl, &dfl);
    pressure_fn(g, p, rr, pr, cr, &fr, &dfr);
    if (df) *df = dfl + dfr;
    return fl + fr + (ur - ul);
}

int orc_exact_star(double g, double rl, double ul, double pl, double rr, double ur, double pr,
                   int method, double* pstar, double* ustar) {
    if (!(g > 1.0) || !(rl > 0.0) || !(rr > 0.0) || !(pl > 0.0) || !(pr > 0.0)) return -1;
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    /* vacuum is generated when the pressure-positivity condition fails */
    if (!(2.0 * (cl + cr) / (g - 1.0) > ur - ul)) return -1;

    double p;
    if (method == 0) {
        double guess = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr);
        p = guess > 1e-8 * (pl < pr ? pl : pr) ? guess : 1e-8 * (pl < pr ? pl : pr);
        /* stop when the relative update reaches round-off; near vacuum the
         * last iterates can wobble by a few ulp, which is accepted */
        double change = 1.0;
        for (int it = 0; it < 500 && change >= 1e-15; ++it) {
            double df;
            double f = total_fn(g, p, rl, ul, pl, cl, rr, ur, pr, cr, &df);
            double pn = p - f / df;
            if (pn <= 0.0) pn = 0.5 * p;
            change = fabs(pn - p) / (0.5 * (pn + p));
            p = pn;
        }
        if (!(change < 1e-12)) return -1;
    } else {
        /* f is increasing in p and f(0) < 0 without vacuum: bracket and halve */
        double lo = 0.0, hi = pl > pr ? pl : pr;
        while (total_fn(g, hi, rl, ul, pl, cl, rr, ur, pr, cr, 0) < 0.0) {
            lo = hi;
            hi *= 2.0;
            if (!isfinite(hi)) return -1;
        }
        for (int it = 0; it < 400; ++it) {
            double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            if (total_fn(g, mid, rl, ul, pl, cl, rr, ur, pr, cr, 0) < 0.0)
                lo = mid;
            else
                hi = mid;
        }
        p = 0.5 * (lo + hi);
    }
    double fl, dfl, fr, dfr;
    pressure_fn(g, p, rl, pl, cl, &fl, &dfl);
    pressure_fn(g, p, rr, pr, cr, &fr, &dfr);
    *pstar = p;
    *ustar = 0.5 * (ul + ur) + 0.5 * (fr - fl);
    return 0;
}

int orc_exact_sample(double g, double rl, double ul, double pl, double rr, double ur, double pr,
                     double xi, double* rho, double* u, double* p) {
    double ps, us;
    if (orc_exact_star(g, rl, ul, pl, rr, ur, pr, 0, &ps, &us)) return -1;
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double gm = (g - 1.0) / (g + 1.0);
    double ex = (g - 1.0) / (2.0 * g);
    if (xi <= us) {
        if (ps > pl) {
            /* left shock with speed from the Rankine-Hugoniot conditions */
            double sl = ul - cl * sqrt((g + 1.0) / (2.0 * g) * ps / pl + ex);
            if (xi <= sl) {
                *rho = rl; *u = ul; *p = pl;
            } else {
                *rho = rl * (ps / pl + gm) / (gm * ps / pl + 1.0);
                *u = us; *p = ps;
            }
        } else {
            double head = ul - cl;
            double tail = us - cl * pow(ps / pl, ex);
            if (xi <= head) {
                *rho = rl; *u = ul; *p = pl;
            } else if (xi >= tail) {
                *rho = rl * pow(ps / pl, 1.0 / g);
                *u = us; *p = ps;
            } else {
                /* inside the left fan: isentropic, with the right-going
                 * Riemann invariant u + 2c/(g-1) of the left state */
                double c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - xi));
                *u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + xi);
                *rho = rl * pow(c / cl, 2.0 / (g - 1.0));
                *p = pl * pow(c / cl, 2.0 * g / (g - 1.0));
            }
        }
    } else {
        if (ps > pr) {
            double sr = ur + cr * sqrt((g + 1.0) / (2.0 * g) * ps / pr + ex);
            if (xi >= sr) {
                *rho = rr; *u = ur; *p = pr;
            } else {
                *rho = rr * (ps / pr + gm) / (gm * ps / pr + 1.0);
                *u = us; *p = ps;
            }
        } else {
            double head = ur + cr;
            double tail = us + cr * pow(ps / pr, ex);
            if (xi >= head) {
                *rho = rr; *u = ur; *p = pr;
            } else if (xi <= tail) {
                *rho = rr * pow(ps / pr, 1.0 / g);
                *u = us; *p = ps;
            } else {
                double c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - xi));
                *u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + xi);
                *rho = rr * pow(c / cr, 2.0 / (g - 1.0));
                *p = pr * pow(c / cr, 2.0 * g / (g - 1.0));
            }
        }
    }
    return 0;
}
