"""Closed-form solution of the impulsively rotated cylinder (App. D, the
axisymmetric viscous flow around a cylinder of radius R that starts rotating
at rate Omega in fluid at rest), nondimensional: r* = r/R, t* = nu t/R^2,
omega* = omega/Omega, u* = u_theta/(Omega R).  Vorticity and velocity as
integrals over Bessel functions of the first and second kind (the form with a
non-oscillatory integrand decaying like exp(-x^2 t*)); evaluated by adaptive
quadrature.  Checked in the tests: u*(1, t*) = 1 (no slip) and the total
vorticity equals the circulation change 2 pi [r u*] (Stokes)."""
import numpy as np
from scipy import integrate, special


def _den(x):
    return special.j1(x) ** 2 + special.y1(x) ** 2


def omega_star(r, t):
    f = lambda x: ((special.j0(x * r) * special.y1(x) - special.j1(x) * special.y0(x * r)) / _den(x)
                   * np.exp(-x * x * t))
    return 2.0 / np.pi * integrate.quad(f, 0.0, np.inf, limit=400)[0]


def u_star(r, t):
    f = lambda x: ((special.j1(x * r) * special.y1(x) - special.j1(x) * special.y1(x * r)) / _den(x)
                   * np.exp(-x * x * t) / x)
    return 1.0 / r + 2.0 / np.pi * integrate.quad(f, 0.0, np.inf, limit=400)[0]


def omega_field(r, t, samples=400, r_max=None):
    """omega* at many radii r >= 1: quadrature on a fine radial grid, cubic
    interpolation between (the field is smooth for t* > 0)."""
    r = np.asarray(r, dtype=np.float64)
    hi = float(r.max()) if r_max is None else r_max
    rs = np.linspace(1.0, max(hi, 1.0 + 1e-9), samples)
    ws = np.array([omega_star(x, t) for x in rs])
    from scipy.interpolate import CubicSpline
    return CubicSpline(rs, ws)(np.clip(r, 1.0, rs[-1]))
