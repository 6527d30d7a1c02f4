"""Pins of the oracle's Newton ICP (Sec. 4.1: a second-order ICP with Newton's
method at each step, the Hessian from the multicomplex step of eq.
csfd_hessian, no small-angle approximation).

The objective of a pass is E(delta) = sum r(exp(delta) T)^2, with the pass's
correspondences held fixed (solver 1: the looked-up model point and normal
are constants of the pass) or differentiated through the projective
association (solver 2).  Its gradient (6 complex-step runs) and Hessian (21
bicomplex runs) are pinned by:

* held correspondences: the gradient is exactly twice the Gauss-Newton
  right-hand side sum J r (J = [p x m; m] is the residual's derivative when
  the correspondence is fixed), and the Hessian is twice sum J J^T plus the
  residual-weighted curvature of the exponential map;
* through the association: central finite differences of the real E
  (gradient; minimum over a step sweep <= 1e-6 relative, runs whose
  correspondence count changes discarded) and of the complex-step gradient
  (Hessian, <= 1e-5);
* one Newton step from near the solution converges quadratically;
* the planar special case: at the true pose of an analytic planar scene the
  residuals vanish and the bilinear model point moves within its plane, so
  the gradient is 0 and the Hessian equals twice the Gauss-Newton matrix
  sum J J^T (J = [p x m; m]);
* Newton tracking (both objectives) recovers a known motion from analytic
  planar model maps to 1e-9, as Gauss-Newton does.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
import scenegen as sg
from test_oracle_icp import CAM, H, W, cfg, coplanar_blocks, planar_scene, twist

MOTION = np.array([0.01, -0.02, 0.015, 0.02, -0.01, 0.03])


def _setup(noisy_model=False):
    sc = planar_scene()
    Tprev = sg.look_at((0.9, 0.2, -1.2), (0, sc.floor_y + 0.2, 0))
    Tcur = expm(twist(MOTION)) @ Tprev
    s = O.seed(0)
    z, _, _ = sg.render_maps(sc, Tcur, W, H, **CAM)
    zm, Pm, Nm = sg.render_maps(sc, Tprev, W, H, **CAM)
    valid = coplanar_blocks(zm, Pm, Nm) if not noisy_model else (zm > 0)
    model = dict(V=Pm[..., None], N=Nm[..., None], Z=zm, valid=valid.astype(np.uint8))
    cur = O.measure(cfg(), s, z)[0]
    return cur, model, Tprev, Tcur, z


@pytest.mark.parametrize("through", [False, True])
def test_planar_true_pose_gradient_zero_hessian_is_twice_gauss_newton(through):
    cur, model, Tprev, Tcur, _ = _setup()
    E, g, Hm, cnt = O.icp_energy(cfg(), 0, cur, model, Tprev, Tcur, through=through)
    assert cnt > 0.5 * W * H
    assert E < 1e-20
    A, b, c2, _ = O.icp_reduce(cfg(), O.seed(0), 0, cur, model, Tprev[..., None], Tcur[..., None])
    assert c2 == cnt
    Af = np.zeros((6, 6))
    iu = np.triu_indices(6)
    Af[iu] = A[:, 0]
    Af = Af + np.triu(Af, 1).T
    assert np.abs(g).max() <= 1e-10 * np.abs(Af).max() * 1e-3
    assert np.abs(Hm - 2 * Af).max() <= 1e-12 * np.abs(2 * Af).max()


def _gn(cur, model, Tprev, T):
    A, b, cnt, r2 = O.icp_reduce(cfg(), O.seed(0), 0, cur, model, Tprev[..., None], T[..., None])
    Af = np.zeros((6, 6))
    iu = np.triu_indices(6)
    Af[iu] = A[:, 0]
    return Af + np.triu(Af, 1).T, b[:, 0], cnt, r2


@pytest.mark.parametrize("noisy_model", [False, True])
def test_held_correspondences_gradient_is_gauss_newton(noisy_model):
    cur, model, Tprev, Tcur, _ = _setup(noisy_model)
    T1 = expm(twist(0.3 * MOTION)) @ Tprev
    E, g, Hm, cnt = O.icp_energy(cfg(), 0, cur, model, Tprev, T1)
    A, b, c2, r2 = _gn(cur, model, Tprev, T1)
    assert cnt == c2 and abs(E - r2) <= 1e-12 * r2
    assert np.abs(g - 2 * b).max() <= 1e-12 * np.abs(2 * b).max()
    # the rest of the Hessian is the residual-weighted curvature of exp: small
    # against the Gauss-Newton part, symmetric
    assert np.abs(Hm - 2 * A).max() <= 0.05 * np.abs(2 * A).max()
    assert np.abs(Hm - 2 * A).max() > 0.0
    assert np.all(np.linalg.eigvalsh(Hm) > 0)


@pytest.mark.parametrize("noisy_model", [False, True])
def test_gradient_and_hessian_match_finite_differences(noisy_model):
    cur, model, Tprev, Tcur, _ = _setup(noisy_model)
    T1 = expm(twist(0.3 * MOTION)) @ Tprev        # away from the solution: residuals nonzero
    E1, g1, H1, c1 = O.icp_energy(cfg(), 0, cur, model, Tprev, T1, through=True)
    assert E1 > 1e-6
    # gradient vs central differences of the real objective
    best = np.inf
    for d in (1e-5, 3e-6, 1e-6, 3e-7, 1e-7):
        fd, same = np.zeros(6), True
        for a in range(6):
            e = np.zeros(6)
            e[a] = d
            Ep = O.icp_energy(cfg(), 0, cur, model, Tprev, expm(twist(e)) @ T1, order=0)
            Em = O.icp_energy(cfg(), 0, cur, model, Tprev, expm(twist(-e)) @ T1, order=0)
            same = same and Ep[3] == c1 and Em[3] == c1
            fd[a] = (Ep[0] - Em[0]) / (2 * d)
        if same:
            best = min(best, np.abs(fd - g1).max() / np.abs(g1).max())
    assert best <= 1e-6, best
    # Hessian vs central differences of the complex-step gradient
    best = np.inf
    for d in (1e-5, 1e-6, 1e-7):
        fd = np.zeros((6, 6))
        for a in range(6):
            e = np.zeros(6)
            e[a] = d
            gp = O.icp_energy(cfg(), 0, cur, model, Tprev, expm(twist(e)) @ T1, order=1, through=True)[1]
            gm = O.icp_energy(cfg(), 0, cur, model, Tprev, expm(twist(-e)) @ T1, order=1, through=True)[1]
            fd[:, a] = (gp - gm) / (2 * d)
        # the left increment's Hessian is symmetric; central differences of the
        # gradient along the left-perturbed pose agree with it to second order
        fds = 0.5 * (fd + fd.T)
        best = min(best, np.abs(fds - H1).max() / np.abs(H1).max())
    assert best <= 1e-5, best
    assert np.abs(H1 - H1.T).max() == 0.0                    # assembled symmetric
    assert np.all(np.linalg.eigvalsh(H1) > 0)


def test_newton_step_near_the_solution_is_quadratic():
    """From a pose close to the solution one Newton step (-H^-1 g with the
    complex-step gradient and Hessian) leaves an error proportional to the
    square of the starting error: halving the start quarters the result."""
    cur, model, Tprev, Tcur, _ = _setup()
    res = []
    for f in (0.05, 0.025):
        T1 = expm(twist(f * MOTION)) @ Tcur
        E, g, Hm, cnt = O.icp_energy(cfg(), 0, cur, model, Tprev, T1)
        assert np.all(np.linalg.eigvalsh(Hm) > 0)
        T2 = expm(twist(-np.linalg.solve(Hm, g))) @ T1
        res.append((np.linalg.norm(T1[:3, 3] - Tcur[:3, 3]), np.linalg.norm(T2[:3, 3] - Tcur[:3, 3])))
    (e0a, e1a), (e0b, e1b) = res
    assert e1a < 0.01 * e0a and e1b < 0.01 * e0b
    assert 3.0 < e1a / e1b < 5.5, (e1a, e1b)


def test_newton_tracking_recovers_known_motion():
    cur, model, Tprev, Tcur, z = _setup()
    out = {}
    for solver in (0, 1, 2):
        for iters in ((3, 0, 0), (10, 5, 4)):
            T, lost, cnt, r2 = O.track(cfg(solver=solver, iters=iters), O.seed(0), z, None, model,
                                       Tprev[..., None], Tprev[..., None])
            assert lost == 0
            out[(solver, iters)] = np.linalg.norm(T[:3, 3, 0] - Tcur[:3, 3])
    for solver in (0, 1, 2):
        assert out[(solver, (10, 5, 4))] < 1e-9
        assert out[(solver, (3, 0, 0))] < 1e-6


def test_newton_needs_a_real_run():
    cur, model, Tprev, Tcur, z = _setup()
    for solver in (1, 2):
        with pytest.raises(ValueError):
            O.track(cfg(solver=solver), O.seed(1, O.P_TRUNC), z, None, model, O.lift(Tprev, O.seed(1)),
                    O.lift(Tprev, O.seed(1)))
