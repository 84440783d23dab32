"""Relaxation-time ratios of Maxwell molecules from the Wang-Chang--Uhlenbeck eigenvalues with
the exact inverse-fifth-power collision kernel (Sec. 2.1, eq:WCU and the eigenvalue passage
around it; Table 4 gives the ratios for one kernel average, see below).

For molecules repelling with a force ~ r^-5 the linearised collision operator has the Burnett
functions as eigenfunctions, with eigenvalues that are kernel averages

    lambda_{r l} ~ < 1 + d_{r0} d_{l0} - x^(r + l/2) P_l(sqrt x) - s^(r + l/2) P_l(sqrt s) >,
    x = cos^2(chi/2),  s = sin^2(chi/2),

taken over the deflection angle chi with the weight of the collision kernel: for this force
law the kernel is b db depsilon, so <F> = int_0^inf F(chi(a)) a da in the dimensionless impact
parameter a.  The SMRT part (n, m) of Hermite order n relaxes with lambda_{m, n-2m}, and
tau*_nm = tau_nm / tau_20 = lambda_{0,2} / lambda_{m, n-2m}.

The deflection of an inverse-power repulsion with force index nu = 5 (potential ~ r^-4) is
chi(a) = pi - 2 theta_0(a) with

    theta_0 = int_0^{x0} dx / sqrt(1 - x^2 - (x / a)^4 / 2),

x0 the positive root of the radicand.  With y = x^2 the radicand is
(y0 - y)(y + y1) / (2 a^4), y0 = a^4 (sqrt(1 + 2/a^4) - 1), y1 = a^4 (sqrt(1 + 2/a^4) + 1),
and x = sqrt(y0) sin(phi) turns theta_0 into the smooth integral
int_0^{pi/2} sqrt(2) a^2 / sqrt(y0 sin^2 phi + y1) dphi, done here by Gauss-Legendre.

Table 4's ratios follow from the same eigenvalues with <sin^4 chi> / <sin^2 chi> = 7/9; the
exact kernel gives 0.631, which changes tau*_40, tau*_50 and tau*_51 only (every other ratio
is a kernel-independent rational).  Host-side set-up of a relaxation table: nothing here runs
in the time step.
"""
import math

import numpy as np
from numpy.polynomial.legendre import leggauss, legval

# Gauss-Legendre panels of the impact-parameter integral: the integrand falls like a^-7
# beyond a ~ 2, so [0, 128] holds it to ~1e-14.
_PANELS = (0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 16.0, 32.0, 128.0)


def deflection_angle(a, n_phi=64):
    """Deflection chi of an r^-5 repulsion at dimensionless impact parameter(s) a > 0."""
    a = np.asarray(a, dtype=float)
    a4 = a ** 4
    root = np.sqrt(1.0 + 2.0 / a4)
    y0 = a4 * (root - 1.0)
    y1 = a4 * (root + 1.0)
    t, w = leggauss(n_phi)
    phi = 0.25 * math.pi * (t + 1.0)
    wphi = 0.25 * math.pi * w
    s2 = np.sin(phi) ** 2
    integrand = np.sqrt(2.0) * a[..., None] ** 2 / np.sqrt(y0[..., None] * s2 + y1[..., None])
    return math.pi - 2.0 * np.sum(wphi * integrand, axis=-1)


def kernel_average(F, n=96):
    """<F> = int_0^inf F(chi(a)) a da for a function F of the deflection angle."""
    t, w = leggauss(n)
    total = 0.0
    for lo, hi in zip(_PANELS[:-1], _PANELS[1:]):
        a = 0.5 * (hi - lo) * (t + 1.0) + lo
        total += float(np.sum(0.5 * (hi - lo) * w * F(deflection_angle(a)) * a))
    return total


def collision_integral_A(l):
    """A_l(5) = int_0^inf (1 - cos^l chi) a da (the inverse-power collision integrals)."""
    return kernel_average(lambda chi: 1.0 - np.cos(chi) ** l)


def eigenvalue(r, l):
    """lambda_{r l} of the linearised operator for Maxwell molecules, up to the common factor."""
    coef = [0.0] * l + [1.0]

    def F(chi):
        x = np.cos(0.5 * chi) ** 2
        s = np.sin(0.5 * chi) ** 2
        return (1.0 + (1.0 if (r == 0 and l == 0) else 0.0) - x ** (r + 0.5 * l) * legval(np.sqrt(x), coef)
                - s ** (r + 0.5 * l) * legval(np.sqrt(s), coef))
    return kernel_average(F)


def tau_star_exact_kernel(N=5):
    """{(n, m): tau_nm / tau_20} for 2 <= n <= N from the exact r^-5 kernel; (2, 1) is 1 (its
    part is identically zero: lambda_{1,0} = 0 by energy conservation)."""
    lam20 = eigenvalue(0, 2)
    out = {}
    for n in range(2, N + 1):
        for m in range(n // 2 + 1):
            out[(n, m)] = 1.0 if (n, m) == (2, 1) else lam20 / eigenvalue(m, n - 2 * m)
    return out
