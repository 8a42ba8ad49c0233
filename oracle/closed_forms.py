"""Closed-form results used to pin the oracle.  Test infrastructure only.

* e+e- -> gamma* -> mu+mu- (massless QED): spin-averaged |M|^2 = e^4 (1 + cos^2 theta),
  sigma = 4 pi alpha^2 / (3 s)  (e.g. Peskin & Schroeder eq. 5.13 and 5.14).
* gg -> Q Qbar at LO (B. L. Combridge, Nucl. Phys. B151 (1979) 429; R. K. Ellis,
  W. J. Stirling, B. R. Webber, "QCD and collider physics", heavy-quark
  production table):
    avg |M|^2 = g^4 [1/(6 t1 t2) - 3/8] [t1^2 + t2^2 + rho - rho^2/(4 t1 t2)],
    t1 = 2 p1.p3 / s, t2 = 2 p2.p3 / s, rho = 4 m^2 / s,
  and the partonic cross section
    sigma = pi alpha_s^2 / (3 s) [(1 + rho + rho^2/16) ln((1+beta)/(1-beta))
                                  - beta (7/4 + 31 rho / 16)],  beta = sqrt(1 - rho).
* massless n-body phase-space volume: see phase_space.massless_volume.
"""
import math

GEV2_TO_PB = 0.3893793721e9   # (hbar c)^2 in pb GeV^2 (PDG)


def ee_mumu_me(cos_theta, alpha):
    e4 = (4.0 * math.pi * alpha) ** 2
    return e4 * (1.0 + cos_theta * cos_theta)


def ee_mumu_sigma(s, alpha):
    return 4.0 * math.pi * alpha * alpha / (3.0 * s)


def gg_tt_me(tau1, s, m, alpha_s):
    g4 = (4.0 * math.pi * alpha_s) ** 2
    tau2 = 1.0 - tau1
    rho = 4.0 * m * m / s
    return g4 * (1.0 / (6.0 * tau1 * tau2) - 3.0 / 8.0) * (
        tau1 * tau1 + tau2 * tau2 + rho - rho * rho / (4.0 * tau1 * tau2))


def gg_tt_me_costheta(c, s, m, alpha_s):
    """Same, as a function of the c.m. angle between the top and the +z gluon."""
    beta = math.sqrt(1.0 - 4.0 * m * m / s)
    return gg_tt_me(0.5 * (1.0 - beta * c), s, m, alpha_s)


def gg_tt_sigma(s, m, alpha_s):
    rho = 4.0 * m * m / s
    beta = math.sqrt(1.0 - rho)
    return math.pi * alpha_s ** 2 / (3.0 * s) * (
        (1.0 + rho + rho * rho / 16.0) * math.log((1.0 + beta) / (1.0 - beta))
        - beta * (7.0 / 4.0 + 31.0 * rho / 16.0))
