"""Full algorithm (Sec. 5.5): the state (omega, Gamma_k) is advanced by a
low-storage third-order Runge-Kutta scheme (Williamson's 2N-storage form);
every stage reconstructs the velocity, evaluates the transport right-hand side
and the Kelvin circulation rates.

Williamson's third-order coefficients (the paper cites the scheme without
printing them):  A = (0, -5/9, -153/128),  B = (1/3, 15/16, 8/15);
    Q <- A_s Q + dt * rhs(state);   state <- state + B_s Q.

Time step (App. B): with the RK3 stability region approximated by the
triangle (C, r) in {(0,0), (1.620,0), (0,0.314)}, C = a_max dt / h and
r = nu dt / h^2, the ray C/r = Re_h leaves the triangle at
dt_max = 1 / (a_max / (1.620 h) + nu / (0.314 h^2)).
"""
from __future__ import annotations

import numpy as np

from . import transport
from .reconstruct import Reconstructor

RK_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)


def rk3_williamson(state, rhs, dt):
    """One low-storage RK3 step of dy/dt = rhs(y, stage) for a list of arrays."""
    state = [np.array(y, dtype=np.float64, copy=True) for y in state]
    Q = [np.zeros_like(y) for y in state]
    for s in range(3):
        r = rhs(state, s)
        for q in range(len(state)):
            Q[q] = RK_A[s] * Q[q] + dt * r[q]
            state[q] = state[q] + RK_B[s] * Q[q]
    return state


def rk3_stage_times():
    """Times of the three stages within a step, in units of dt: the same
    recurrences applied to the time itself (d t / d t = 1)."""
    t, q, c = 0.0, 0.0, []
    for s in range(3):
        c.append(t)
        q = RK_A[s] * q + 1.0
        t = t + RK_B[s] * q
    return c


def dt_max(h, nu, a_max):
    return 1.0 / (a_max / (1.620 * h) + nu / (0.314 * h * h))


class Stepper:
    def __init__(self, geom, lgf_tab=None, method="direct"):
        self.geom = geom
        self.rec = Reconstructor(geom, lgf_tab=lgf_tab)
        self.nu = geom.grid.nu
        self.method = method
        if method == "direct":
            self._lu = None

    def _solve(self, omega, Gamma, x0=None):
        R = self.rec
        if self.method == "direct":
            import scipy.linalg as sla
            if self._lu is None:
                self._lu = sla.lu_factor(R.dense_matrix())
            b = R.rhs(omega, Gamma)
            x = sla.lu_solve(self._lu, b)
            return x, b, {"iters": 0}
        return R.solve(omega, Gamma, method="gmres", x0=x0)

    def stage(self, omega, Gamma, x0=None):
        x, b, info = self._solve(omega, Gamma, x0=x0)
        rec = self.rec.recover(omega, x)
        dw, dG, wb, _ = transport.rhs(self.geom, omega, rec.U, rec.V, self.nu)
        return dw, dG, rec, x, info

    def set_motion(self, motions):
        """Rigid motion (u_x, u_y, omega) of every body from now on."""
        self.geom.set_rigid_motion(motions)
        self.rec.psib_t = self.geom.psi_tilde_b()

    def step(self, omega, Gamma, dt, record=None, motion=None, t=0.0):
        """One RK3 step from time t; motion: optional function of time giving
        the rigid motion of every body, applied at each stage's time."""
        omega = np.where(self.geom.fluid, omega, 0.0)
        last = {"x": None}
        c = rk3_stage_times()

        def rhs(state, s):
            if motion is not None:
                self.set_motion(motion(t + c[s] * dt))
            w, G = state
            dw, dG, rec, x, info = self.stage(w, G, x0=last["x"])
            last["x"] = x
            if record is not None:
                record.append((w.copy(), G.copy(), rec, info))
            return [dw, dG]

        omega, Gamma = rk3_williamson([omega, Gamma], rhs, dt)
        return omega, Gamma
