"""Pins of the oracle's optional terms (the applications of Sec. 6): slide DOFs
and 6-DOF floating roots, the drag potential and the penalty frictional contact
of Eq. FRI at discrete points.

Each test compares the oracle with something that is not the oracle: the exact
discrete trajectory of a free body (the position-based step reproduces a
parabola exactly, and drag gives a closed-form velocity decay), the pairwise
form of App. A for the drag term, closed forms and a scalar root solve of a
point mass landing on the plane, hand-built transforms for slides, and central
differences of the objective and of the gradient.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle.oracle import Oracle
from paper_1709_04145_amd import workloads as W

G = np.array([0.0, 0.0, -9.81])


def _free_body(mm, gravity=G, drag=None, contacts=(), plane=(0.0, 0.0, 1.0, 0.0), d1=0.0, d2=0.0, kinds=None,
               axes=None):
    """One model: a single link on a floating root (3 slides, 3 hinges) by default."""
    kinds = W.FREE_KINDS if kinds is None else np.asarray(kinds, np.int32)
    axes = W.FREE_AXES if axes is None else np.asarray(axes, np.float64)
    model = dict(parent=np.array([-1]), dofs=np.array([len(kinds)], np.int32), axis=axes,
                 offset=np.zeros((1, 3)), mm=np.asarray(mm, np.float64)[None, :])
    return W._with_extras([model], kinds=[kinds], drag=None if drag is None else [np.array([drag])],
                          contacts=[[(0, p) for p in contacts]], gravity=gravity, plane=plane, d1=d1, d2=d2)


def _box():
    return W.box_mass_moment(0.6, 0.2, 800.0)  # centre of mass off the link origin


def test_free_body_falls_on_the_exact_parabola():
    """A rigid body that does not rotate: the minimizer of the step keeps the
    orientation and moves the origin by 2 t_k - t_{k-1} + dt^2 g exactly."""
    d = _free_body(_box())
    orc = Oracle(d)
    dt = 0.05
    qc = np.array([0.3, -0.2, 1.0, 0.4, -0.7, 1.1])
    qp = qc - np.array([0.02, 0.05, -0.01, 0.0, 0.0, 0.0])
    q, st = orc.step(qp, qc, dt, tol=1e-12, max_iter=200)
    assert st["flag"][0] == 1
    np.testing.assert_allclose(q[:3], 2 * qc[:3] - qp[:3] + dt * dt * G, rtol=0, atol=1e-12)
    np.testing.assert_allclose(q[3:], qc[3:], rtol=0, atol=1e-12)


@pytest.mark.parametrize("c", [0.05, 0.5])
def test_drag_decays_the_velocity_by_one_over_one_plus_two_c(c):
    """No gravity, a non-rotating body with drag c: the step's stationarity
    m (t - 2 t_k + t_{k-1}) + 2 c m (t - t_k) = 0 gives t - t_k = (t_k - t_{k-1}) / (1 + 2c)."""
    d = _free_body(_box(), gravity=[0.0, 0.0, 0.0], drag=c)
    orc = Oracle(d)
    qc = np.array([0.3, -0.2, 1.0, 0.4, -0.7, 1.1])
    v = np.array([0.03, -0.02, 0.05, 0.0, 0.0, 0.0])
    q, st = orc.step(qc - v, qc, 0.05, tol=1e-12, max_iter=200)
    assert st["flag"][0] == 1
    np.testing.assert_allclose(q - qc, v / (1.0 + 2.0 * c), rtol=0, atol=1e-12)


def test_drag_pairwise_form_of_appendix_A_differs_by_a_constant():
    """App. A writes the drag integral as c (I(q,q) - 2 I(q,q_k) + I(q_k,q_k)):
    the oracle's I-form with it and its D-form objective differ by a
    q-independent constant (contacts switched off: they are not an I-combination)."""
    d = W.random_extras_models(6, 160, max_links=5)
    d.contact_link = d.contact_point = None
    orc = Oracle(d)
    rng = np.random.default_rng(161)
    qp, qc = (rng.uniform(-1, 1, d.n_dofs) for _ in range(2))
    diffs = []
    for _ in range(3):
        q = rng.uniform(-1, 1, d.n_dofs)
        E, _, S = orc.objective_grad(q, qp, qc, 0.03)
        diffs.append(E - orc.objective_Iform(q, qp, qc, 0.03))
    scale = np.max(np.abs(diffs)) + 1.0
    assert np.max(np.abs(diffs[1] - diffs[0])) <= 1e-12 * scale
    assert np.max(np.abs(diffs[2] - diffs[0])) <= 1e-12 * scale
    # and the drag terms are not zero: removing them changes the q-dependence
    d.drag = None
    orc0 = Oracle(d)
    q = rng.uniform(-1, 1, d.n_dofs)
    assert np.max(np.abs(orc0.objective_grad(q, qp, qc, 0.03)[0] - orc.objective_grad(q, qp, qc, 0.03)[0])) > 1e-3


def _point_mass(m, contacts, d1, d2, plane=(0.0, 0.0, 1.0, 0.0)):
    """A translating point-like body: three slides, mass m concentrated at the origin."""
    mm = np.zeros(10)
    mm[9] = m
    return _free_body(mm, contacts=contacts, d1=d1, d2=d2, plane=plane, kinds=[1, 1, 1], axes=np.eye(3))


def test_point_mass_landing_matches_the_closed_form():
    """Three slides, mass m at the origin, one contact point there, no friction:
    where it penetrates, m (z - c) - dt^2 m g_z - 2 dt^2 D1 (h - z) = 0 with
    c = 2 z_k - z_{k-1}, so z = (m c + dt^2 m g_z + 2 dt^2 D1 h) / (m + 2 dt^2 D1);
    x, y follow the free parabola."""
    m, d1, dt, h = 1.7, 3.0e4, 0.01, 0.02
    d = _point_mass(m, [[0.0, 0.0, 0.0]], d1, 0.0, plane=(0.0, 0.0, 1.0, h))
    orc = Oracle(d)
    qc = np.array([0.1, 0.2, 0.021])
    qp = qc - np.array([0.01, -0.02, -0.015])
    q, st = orc.step(qp, qc, dt, tol=1e-13, max_iter=200)
    assert st["flag"][0] == 1
    c = 2 * qc - qp
    z = (m * c[2] + dt * dt * m * G[2] + 2 * dt * dt * d1 * h) / (m + 2 * dt * dt * d1)
    assert z < h
    np.testing.assert_allclose(q, [c[0], c[1], z], rtol=0, atol=1e-12)


def test_point_mass_sliding_with_friction_matches_a_scalar_root():
    """With friction (D2 > 0) and a tangential velocity the step couples x and z:
    m (x - c_x) + 2 D2 d^2 (x - x_k) = 0 gives x(z); then z solves
    m (z - c_z) - dt^2 m g_z - 2 d (dt^2 D1 + D2 (x - x_k)^2) = 0, d = h - z
    (a scalar root, brentq)."""
    m, d1, d2, dt, h = 1.3, 2.0e4, 4.0e5, 0.01, 0.0
    d = _point_mass(m, [[0.0, 0.0, 0.0]], d1, d2)
    orc = Oracle(d)
    qc = np.array([0.5, -0.1, -0.004])
    qp = qc - np.array([0.012, 0.0, -0.003])
    q, st = orc.step(qp, qc, dt, tol=1e-13, max_iter=500)
    assert st["flag"][0] == 1
    c = 2 * qc - qp

    def x_of(z):
        w = 2 * d2 * (h - z) ** 2
        return (m * c[0] + w * qc[0]) / (m + w)

    def fz(z):
        dd = h - z
        return m * (z - c[2]) - dt * dt * m * G[2] - 2 * dd * (dt * dt * d1 + d2 * (x_of(z) - qc[0]) ** 2)

    z = brentq(fz, -0.1, h - 1e-12, xtol=1e-15, rtol=1e-15)
    np.testing.assert_allclose(q, [x_of(z), c[1], z], rtol=0, atol=1e-11)
    assert abs(q[0] - c[0]) > 1e-6  # friction acted


def test_slides_follow_hand_built_transforms():
    """A hinge about z (angle th) then a child link on a slide along its x axis
    (displacement s): the child's origin is R_z(th) (o + s e_x) and its
    orientation R_z(th)."""
    mm = W.box_mass_moment(0.5, 0.1, 1000.0)
    models = [dict(parent=np.array([-1, 0]), dofs=np.array([1, 1], np.int32),
                   axis=np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]]),
                   offset=np.array([[0.1, 0.2, 0.3], [0.5, 0.0, 0.05]]), mm=np.stack([mm, mm]))]
    d = W._with_extras(models, kinds=[np.array([0, 1], np.int32)])
    th, s = 0.7, 0.33
    P = Oracle(d).poses(np.array([th, s]))
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    np.testing.assert_allclose(P[1][:, :3], Rz, atol=1e-15)
    np.testing.assert_allclose(P[1][:, 3], np.array([0.1, 0.2, 0.3]) + Rz @ np.array([0.5 + s, 0.0, 0.05]),
                               atol=1e-15)


def _active_state(d, seed):
    """A state of random extras models in which many contact points penetrate
    (plane z < -0.2) and move."""
    rng = np.random.default_rng(seed)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.05 * rng.standard_normal(d.n_dofs)
    q = qc + 0.05 * rng.standard_normal(d.n_dofs)
    return q, qp, qc


def _penetrating(orc, d, q):
    P = orc.poses(q)
    x = np.array([P[l] @ np.append(p, 1.0) for l, p in zip(d.contact_link, d.contact_point)])
    return int(np.sum(x[:, 2] < -0.2))


def test_gradient_with_extras_matches_central_differences():
    d = W.random_extras_models(8, 162, max_links=5)
    orc = Oracle(d)
    q, qp, qc = _active_state(d, 163)
    tau = np.random.default_rng(164).uniform(-3, 3, d.n_dofs)
    dt = 0.02
    assert _penetrating(orc, d, q) >= 3  # contact terms active
    _, g, _ = orc.objective_grad(q, qp, qc, dt, tau)
    h = 1e-6
    fd = np.zeros(d.n_dofs)
    do = d.dof_offset
    model_of = np.searchsorted(do, np.arange(d.n_dofs), side="right") - 1
    for j in range(d.n_dofs):
        a, b = q.copy(), q.copy()
        a[j] += h
        b[j] -= h
        i = model_of[j]
        fd[j] = (orc.objective_grad(a, qp, qc, dt, tau)[0][i] - orc.objective_grad(b, qp, qc, dt, tau)[0][i]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7 * np.max(np.abs(g)))


def test_hessian_with_extras_matches_central_differences_of_the_gradient():
    d = W.random_extras_models(6, 172, max_links=4)
    orc = Oracle(d)
    q, qp, qc = _active_state(d, 173)
    dt = 0.02
    assert _penetrating(orc, d, q) >= 3  # contact terms active
    H = orc.hessian(q, qp, qc, dt)
    do = d.dof_offset
    h = 1e-6
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        n = do[i + 1] - do[i]
        fd = np.zeros((n, n))
        for j in range(n):
            a, b = q.copy(), q.copy()
            a[do[i] + j] += h
            b[do[i] + j] -= h
            fd[:, j] = (orc.objective_grad(a, qp, qc, dt)[1][sl] - orc.objective_grad(b, qp, qc, dt)[1][sl]) / (2 * h)
        np.testing.assert_allclose(H[i], fd, rtol=1e-5, atol=1e-6 * max(1.0, np.max(np.abs(fd))))


def test_extras_steps_reach_the_newton_minimizer():
    """Random trees with slides, floating roots, drag and active contact: the
    L-BFGS step ends within the tolerance-implied distance of the minimizer that
    dense Newton (the pinned Hessian) polishes."""
    d = W.random_extras_models(8, 167, max_links=5)
    orc = Oracle(d)
    _, qp, qc = _active_state(d, 168)
    dt = 0.01
    q, st = orc.step(qp, qc, dt, tol=1e-9, max_iter=3000)
    assert np.all(st["flag"] == 1), st
    assert _penetrating(orc, d, q) >= 3  # contact terms active at the minimizer
    qx = q.copy()
    do = d.dof_offset
    for _ in range(4):
        _, g, _ = orc.objective_grad(qx, qp, qc, dt)
        H = orc.hessian(qx, qp, qc, dt)
        for i in range(d.n_models):
            sl = slice(do[i], do[i + 1])
            qx[sl] -= np.linalg.solve(H[i], g[sl])
    _, g, _ = orc.objective_grad(q, qp, qc, dt)
    H = orc.hessian(qx, qp, qc, dt)
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        bound = 1.5 * np.linalg.norm(np.linalg.inv(H[i]), 2) * np.linalg.norm(g[sl])
        assert np.linalg.norm(q[sl] - qx[sl]) <= bound + 1e-12, i


def test_extras_description_is_validated():
    d = W.random_extras_models(2, 169)
    d.drag = -np.abs(d.drag) - 1.0
    with pytest.raises(ValueError):
        Oracle(d)
    d = W.random_extras_models(2, 169)
    d.dof_kind = d.dof_kind.copy()
    d.dof_kind[0] = 2
    with pytest.raises(ValueError):
        Oracle(d)


def test_orders_above_two_reject_extras():
    d = W.random_extras_models(2, 170)
    orc = Oracle(d)
    q = np.zeros(d.n_dofs)
    with pytest.raises(NotImplementedError):
        orc.step_hoc(3, q, q, 0.01)
    with pytest.raises(NotImplementedError):
        orc.step_lm_eq(q, q, 0.01)
