"""Roots of the electrostatic dispersion relation of Maxwellian plasmas,
1 + sum_s n_s / (k^2 s_s^2) (1 + zeta_s Z(zeta_s)) = 0 with
zeta_s = (omega / k - u_s) / sqrt(2 s_s^2) and the plasma dispersion function
Z(zeta) = i sqrt(pi) w(zeta) (w: Faddeeva).  Linear theory fixes the damping
and growth rates the long GPU runs are checked against."""
import math

def root_beams(k, v0, guess):
    """Root omega = (re, im) of the dispersion relation of one Maxwellian
    (v0 = 0) or two unit-variance beams at +-v0 sharing the density."""
    from scipy.special import wofz
    from scipy.optimize import fsolve

    def f(z):
        w = complex(z[0], z[1])
        D = 1.0
        beams = (0.0,) if v0 == 0.0 else (v0, -v0)
        for b in beams:
            zeta = (w / k - b) / math.sqrt(2)
            Z = 1j * math.sqrt(math.pi) * wofz(zeta)
            D += (1 + zeta * Z) / (k * k * len(beams))
        return [D.real, D.imag]

    r = fsolve(f, guess, xtol=1e-13)
    return r[0], r[1]


def root_maxwellians(k, comps, guess):
    """Root of the dispersion relation of a sum of drifting Maxwellians,
    comps = [(density, drift, variance)]."""
    from scipy.special import wofz
    from scipy.optimize import fsolve

    def f(z):
        w = complex(z[0], z[1])
        D = 1.0
        for n, u, s2 in comps:
            zeta = (w / k - u) / math.sqrt(2 * s2)
            Z = 1j * math.sqrt(math.pi) * wofz(zeta)
            D += n / (k * k * s2) * (1 + zeta * Z)
        return [D.real, D.imag]

    r = fsolve(f, guess, xtol=1e-13)
    return r[0], r[1]
