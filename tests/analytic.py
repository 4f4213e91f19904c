"""Closed forms and measurement helpers shared by the physics tests (no
method arithmetic: these evaluate textbook results and read fields)."""
import math

import numpy as np


def miller_scriven_omega2(sigma, R, rho_in, rho_out, nu_in, nu_out):
    """Angular frequency of the l = 2 shape mode of a viscous drop in a viscous
    host (Miller and Scriven, as used in the droplet-oscillation study,
    Eqs. millscriv-millscriv3): the inviscid Lamb frequency with the first
    viscous corrections."""
    den = 2 * rho_out + 3 * rho_in
    w_star = math.sqrt(24 * sigma / (R ** 3 * den))
    alpha = (25 * math.sqrt(nu_in * nu_out) * rho_in * rho_out
             / (math.sqrt(2) * R * den * (math.sqrt(nu_in) * rho_in + math.sqrt(nu_out) * rho_out)))
    return w_star - 0.5 * alpha * math.sqrt(w_star) + 0.25 * alpha ** 2


def axis_radius(rn_line):
    """Interface position on a line through the centre: rho^N = 0 crossings by
    linear interpolation between the adjacent nodes; half the distance between
    the outermost crossings."""
    s = np.sign(rn_line)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    if len(idx) < 2:
        return float("nan")
    xs = [i + rn_line[i] / (rn_line[i] - rn_line[i + 1]) for i in (idx[0], idx[-1])]
    return 0.5 * (xs[1] - xs[0])


def damped_fit(ts, r, w_guess=2 * math.pi / 1000.0):
    """Least-squares fit of R(t) = R_D + b exp(-l t) cos(w t + ph); returns
    (R_D, |w|, l)."""
    from scipy.optimize import curve_fit

    def model(t, a, b, lam, w, ph):
        return a + b * np.exp(-lam * t) * np.cos(w * t + ph)
    p0 = [float(r.mean()), float(r[0] - r.mean()), 1e-4, w_guess, math.pi]
    pp, _ = curve_fit(model, ts, r, p0=p0, maxfev=50000)
    return float(pp[0]), abs(float(pp[3])), float(pp[2])
