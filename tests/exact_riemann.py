"""Exact solution of the Riemann problem of the 1D Euler equations (ideal
gas), written from the standard mathematics (two nonlinear waves separated by
a contact; the star pressure solves f_L(p) + f_R(p) + u_R - u_L = 0 with the
shock / rarefaction branches of f; Newton iteration).  Used to pin the oracle
in its b = 0 limit, where the method reduces to relaxing-TVD hydrodynamics."""
import numpy as np


def _f(p, rho, pk, gamma):
    a = np.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        f = (p - pk) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:       # rarefaction
        f = 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma):
    """(p*, u*) for left/right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, gamma)
        fr, dfr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, gamma, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    al = np.sqrt(gamma * pl / rl)
    ar = np.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3,) + np.shape(xi))
    for idx, s in np.ndenumerate(np.asarray(xi)):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + g1) / (g1 * ps / pl + 1.0))
                sh = ul - al * np.sqrt((gamma + 1.0) / (2 * gamma) * ps / pl + (gamma - 1.0) / (2 * gamma))
                w = (rl, ul, pl) if s < sh else (rs, us, ps)
            else:        # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / gamma)
                ast = al * (ps / pl) ** ((gamma - 1.0) / (2 * gamma))
                head, tail = ul - al, us - ast
                if s < head:
                    w = (rl, ul, pl)
                elif s > tail:
                    w = (rs, us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (al + (gamma - 1.0) / 2.0 * ul + s)
                    c = 2.0 / (gamma + 1.0) * (al + (gamma - 1.0) / 2.0 * (ul - s))
                    r = rl * (c / al) ** (2.0 / (gamma - 1.0))
                    w = (r, u, pl * (c / al) ** (2.0 * gamma / (gamma - 1.0)))
        else:        # right of contact
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + g1) / (g1 * ps / pr + 1.0))
                sh = ur + ar * np.sqrt((gamma + 1.0) / (2 * gamma) * ps / pr + (gamma - 1.0) / (2 * gamma))
                w = (rr, ur, pr) if s > sh else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / gamma)
                ast = ar * (ps / pr) ** ((gamma - 1.0) / (2 * gamma))
                head, tail = ur + ar, us + ast
                if s > head:
                    w = (rr, ur, pr)
                elif s < tail:
                    w = (rs, us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (-ar + (gamma - 1.0) / 2.0 * ur + s)
                    c = 2.0 / (gamma + 1.0) * (ar - (gamma - 1.0) / 2.0 * (ur - s))
                    r = rr * (c / ar) ** (2.0 / (gamma - 1.0))
                    w = (r, u, pr * (c / ar) ** (2.0 * gamma / (gamma - 1.0)))
        out[(slice(None),) + idx] = w
    return out
