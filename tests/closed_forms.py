"""Closed forms used to pin the oracle's forward model (independent of it).

* Convolution of exp(-beta t) with each term of Feng's input (Sec. III-A1):
    exp(-beta t) * exp(-kappa t)   = (e^{-kappa t} - e^{-beta t}) / (beta - kappa)
    exp(-beta t) * t exp(-kappa t) = t e^{-kappa t}/(beta - kappa)
                                     - (e^{-kappa t} - e^{-beta t})/(beta - kappa)^2
  with the beta = kappa limits t e^{-beta t} and t^2 e^{-beta t} / 2.
* RK4 integration of the 2TCM ODE (Eq. (1)) with a piecewise-linear input.
"""
import numpy as np


def _e0(t, beta, kappa):
    if abs(beta - kappa) < 1e-12:
        return t * np.exp(-beta * t)
    return (np.exp(-kappa * t) - np.exp(-beta * t)) / (beta - kappa)


def _e1(t, beta, kappa):
    if abs(beta - kappa) < 1e-12:
        return 0.5 * t * t * np.exp(-beta * t)
    d = beta - kappa
    return t * np.exp(-kappa * t) / d - (np.exp(-kappa * t) - np.exp(-beta * t)) / d ** 2


def feng_conv_exp(t, beta, p):
    """int_0^t exp(-beta (t - s)) C_a(s) ds for Feng's input C_a."""
    t = np.asarray(t, dtype=np.float64)
    return (p["b1"] * _e1(t, beta, p["k1"]) - (p["b2"] + p["b3"]) * _e0(t, beta, p["k1"])
            + p["b2"] * _e0(t, beta, p["k2"]) + p["b3"] * _e0(t, beta, p["k3"]))


def feng_integral(t, p):
    """int_0^t C_a(s) ds (the beta = 0 case)."""
    return feng_conv_exp(t, 0.0, p)


def rk4_2tcm_nodes(theta, cp, h, sub=40):
    """Node TAC of Eq. (1)-(2) (C_wb = C_p) by classical RK4 with `sub` steps
    per grid interval; the input is the straight line between nodes.
    theta = (K1, k2, k3, k4, vB)."""
    K1, k2, k3, k4, vB = theta
    cp = np.asarray(cp, dtype=np.float64)
    K = cp.shape[0] - 1
    out = np.zeros(K + 1)
    y = np.zeros(2)

    def f(yv, c):
        cf, cm = yv
        return np.array([K1 * c - (k2 + k3) * cf + k4 * cm, k3 * cf - k4 * cm])

    dtau = h / sub
    for k in range(K):
        c0, c1 = cp[k], cp[k + 1]
        for s in range(sub):
            a = s / sub
            ca, cmid, cb = c0 + (c1 - c0) * a, c0 + (c1 - c0) * (a + 0.5 / sub), c0 + (c1 - c0) * (a + 1.0 / sub)
            q1 = f(y, ca)
            q2 = f(y + 0.5 * dtau * q1, cmid)
            q3 = f(y + 0.5 * dtau * q2, cmid)
            q4 = f(y + dtau * q3, cb)
            y = y + dtau / 6.0 * (q1 + 2 * q2 + 2 * q3 + q4)
        out[k + 1] = (1 - vB) * (y[0] + y[1]) + vB * c1
    out[0] = vB * cp[0]
    return out


def rk4_reference_nodes(theta, cr, h, sub=40):
    """Node TAC of the lp-ntPET ODE behind Eq. (3)-(4),
        C_t' = R1 C_r' + k2 C_r - (k2a + gamma g(t)) C_t,   C_t(0) = R1 C_r(0),
    by classical RK4 with `sub` steps per grid interval, the reference TAC being
    the straight line between nodes and g(t) the peak-normalised gamma variate
    s^alpha exp(alpha (1 - s)), s = (t - tD)/(tP - tD), zero before tD.
    theta = (R1, k2, k2a, gamma, tD, tP, alpha)."""
    R1, k2, k2a, gam, tD, tP, alpha = theta
    cr = np.asarray(cr, dtype=np.float64)
    K = cr.shape[0] - 1

    def g(t):
        if t <= tD:
            return 0.0
        s = (t - tD) / (tP - tD)
        return s ** alpha * np.exp(alpha * (1.0 - s))

    out = np.zeros(K + 1)
    y = R1 * cr[0]
    out[0] = y
    dtau = h / sub
    for k in range(K):
        c0, c1 = cr[k], cr[k + 1]
        slope = (c1 - c0) / h

        def f(t, yv):
            c = c0 + slope * (t - k * h)
            return R1 * slope + k2 * c - (k2a + gam * g(t)) * yv

        for s in range(sub):
            t = k * h + s * dtau
            q1 = f(t, y)
            q2 = f(t + 0.5 * dtau, y + 0.5 * dtau * q1)
            q3 = f(t + 0.5 * dtau, y + 0.5 * dtau * q2)
            q4 = f(t + dtau, y + dtau * q3)
            y = y + dtau / 6.0 * (q1 + 2 * q2 + 2 * q3 + q4)
        out[k + 1] = y
    return out
