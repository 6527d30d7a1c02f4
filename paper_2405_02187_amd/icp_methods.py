"""Point-to-plane ICP with three optimisers (Sec. 5.1, the comparison of
Fig. 3): gradient descent, nonlinear conjugate gradients and Newton's method.

The source is a depth image measured by the library; the target is the
analytic model of the same scene seen from a reference pose, and the true
pose of the source is a random rigid transform of it.  Every method
minimises the same objective E(T) = sum of squared point-to-plane residuals
(``xslam_icp_energy``: E with its gradient and Hessian in the left increment;
the correspondences are re-associated at every evaluated pose and held fixed
for its derivatives, as ICP does), starting from the reference pose, and
updates T <- exp(alpha d) T along its direction d, a step of at most
``radius`` (rad + m, the norm of alpha d) -- a trust region: the sum over the
correspondences also falls when a step loses them, so an unbounded line
search can walk off the surface:

* ``gd``: d = -g with a backtracking (Armijo) line search;
* ``ncg``: Polak-Ribiere+ conjugate directions, the same line search,
  restarted every 6 iterations or when d is not a descent direction;
* ``newton``: d = -H^-1 g (the complex-step Hessian), full step, halved
  while E does not decrease; the gradient step when H is not positive
  definite or no halving decreases E.  With a
  threshold ``eta`` (Sec. 5.2: Newton's method depends on its start), the
  gradient step is taken instead while E exceeds eta;
* ``gd_fd``: gradient descent on central finite differences of E (step
  ``fd_step``) instead of the complex-step gradient, the comparison the
  paper draws for relocalisation.

The paper runs this on a depth image of ICL-NUIM lr kt1 (not available
here); a seeded synthetic scene stands in for it.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import xslam as X


def _hat(xi):
    M = np.zeros((4, 4))
    M[0, 1], M[0, 2], M[1, 0], M[1, 2], M[2, 0], M[2, 1] = -xi[2], xi[1], xi[2], -xi[0], -xi[1], xi[0]
    M[:3, 3] = xi[3:]
    return M


def se3_exp(xi):
    return expm(_hat(np.asarray(xi, dtype=np.float64)))


def pose_errors(T, T_true):
    dt = float(np.linalg.norm(T[:3, 3] - T_true[:3, 3]))
    Rr = T[:3, :3] @ T_true[:3, :3].T
    ang = float(np.degrees(np.arccos(np.clip((np.trace(Rr) - 1.0) / 2.0, -1.0, 1.0))))
    return dt, ang


class Objective:
    """E, g, H of one ICP pass of `slam` (a context with no directions whose
    measured maps and model maps are set) at pose T."""

    def __init__(self, slam, level: int, through: bool = False):
        self.slam, self.level, self.through, self.evals = slam, level, through, 0

    def __call__(self, T):
        self.slam.set(X.F_POSE, np.asarray(T, dtype=np.float64)[None])
        self.evals += 1
        return self.slam.icp_energy(self.level, self.through)


def _line_search(f, T, E, g, d, alpha0, shrink=0.5, c1=1e-4, max_halvings=40):
    slope = float(g @ d)
    a = alpha0
    for _ in range(max_halvings):
        Tn = se3_exp(a * d) @ T
        En = f(Tn)[0]
        if En <= E + c1 * a * slope:
            return a, Tn
        a *= shrink
    return 0.0, T


def _clip(d, radius):
    n = float(np.linalg.norm(d))
    return d if n <= radius else d * (radius / n)


def _fd_gradient(f, T, h):
    g = np.zeros(6)
    for a in range(6):
        e = np.zeros(6)
        e[a] = h
        g[a] = (f(se3_exp(e) @ T)[0] - f(se3_exp(-e) @ T)[0]) / (2.0 * h)
    return g


def optimise(f, T_start, T_true, method: str, iters: int = 30, radius: float = 0.05, eta=None,
             fd_step: float = 1e-3):
    """-> list of per-iteration dict(it, E, t_err_m, r_err_deg, count, step)
    (step: the direction taken to reach the next iterate, "newton" or
    "gradient")."""
    T = np.array(T_start, dtype=np.float64)
    E, g, H, cnt = f(T)
    if method == "gd_fd":
        g = _fd_gradient(f, T, fd_step)
    trace = []
    d_prev, g_prev, alpha = None, None, 1.0
    for it in range(iters + 1):
        dt, dr = pose_errors(T, T_true)
        trace.append(dict(it=it, E=float(E), t_err_m=dt, r_err_deg=dr, count=int(cnt)))
        if it == iters or not np.isfinite(E) or np.linalg.norm(g) == 0.0:
            break
        newton = method == "newton" and (eta is None or E <= eta)
        Tn = None
        if newton:
            try:
                np.linalg.cholesky(H)
                d = -np.linalg.solve(H, g)
            except np.linalg.LinAlgError:
                d = None
            if d is not None:
                d = _clip(d, radius)
                a = 1.0
                for _ in range(20):
                    Tc = se3_exp(a * d) @ T
                    if f(Tc)[0] <= E:
                        Tn = Tc
                        break
                    a *= 0.5
            trace[-1]["step"] = "newton" if Tn is not None else "gradient"
        else:
            trace[-1]["step"] = "gradient"
        if Tn is None:
            # gradient descent / nonlinear CG, and the fall-back of a Newton
            # step that is not a descent step
            d = -g
            if method == "ncg" and d_prev is not None and it % 6 != 0:
                beta = max(0.0, float(g @ (g - g_prev)) / float(g_prev @ g_prev))
                d = -g + beta * d_prev
                if float(g @ d) >= 0.0:
                    d = -g
            # initial step: twice the last accepted one, within the radius
            a0 = alpha * 2.0 if d_prev is not None else 1.0 / max(np.linalg.norm(g), 1e-300)
            a0 = min(a0, radius / max(float(np.linalg.norm(d)), 1e-300))
            alpha, Tn = _line_search(f, T, E, g, d, a0)
            if alpha == 0.0:
                break            # no sufficient decrease along d: stationary
            d_prev, g_prev = d, g
        T = Tn
        E, g, H, cnt = f(T)
        if method == "gd_fd":
            g = _fd_gradient(f, T, fd_step)
    return trace


def run(slam, level: int, T_ref, T_true, iters: int = 30, methods=("gd", "ncg", "newton"), radius: float = 0.05,
        through: bool = False) -> dict:
    """The three optimisers from the reference pose.  `slam` holds the
    measured maps of the source depth and the model maps at T_ref (with
    XSLAM_F_PREV_POSE = T_ref as the projection reference)."""
    f = Objective(slam, level, through)
    out = {}
    for m in methods:
        f.evals = 0
        out[m] = dict(trace=optimise(f, T_ref, T_true, m, iters, radius), evaluations=f.evals)
    return out
