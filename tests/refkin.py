"""Independent reference kinematics for pinning the oracle (test-only).

Rotations come from scipy (rotation vectors), body integrals from tensor-product
Gauss-Legendre cubature over each box, and velocities of body points from the
textbook world-frame Jacobian  dx/dq_n = w_n x (x - p_n).  Nothing here calls
the oracle's arithmetic.
"""
import numpy as np
from scipy.spatial.transform import Rotation


def link_frames(desc, q):
    """World transforms (4x4) of every link, and per DOF the world axis and joint point."""
    L = desc.n_links
    T = np.zeros((L, 4, 4))
    w_axis = np.zeros((desc.n_dofs, 3))
    p_joint = np.zeros((desc.n_dofs, 3))
    dof_start = desc.link_dof_start
    for i in range(desc.n_models):
        lo, hi = desc.link_offset[i], desc.link_offset[i + 1]
        for l in range(lo, hi):
            par = desc.parent[l]
            Tp = np.eye(4) if par < 0 else T[lo + par]
            R = Tp[:3, :3].copy()
            t = Tp[:3, :3] @ desc.offset[l] + Tp[:3, 3]
            for k in range(desc.dofs_per_link[l]):
                n = dof_start[l] + k
                a = desc.axis[n] / np.linalg.norm(desc.axis[n])
                w_axis[n] = R @ a
                p_joint[n] = t
                R = R @ Rotation.from_rotvec(a * q[n]).as_matrix()
            T[l, :3, :3] = R
            T[l, :3, 3] = t
            T[l, 3, 3] = 1.0
    return T, w_axis, p_joint


def box_dims_from_moment(mm_row):
    """Recover (L, w, rho) of the generator's box from its mass moment row."""
    m = mm_row[9]
    L = 2.0 * mm_row[3] / m
    w = np.sqrt(12.0 * mm_row[4] / m)
    rho = m / (L * w * w)
    return L, w, rho


def box_cubature(L, w, npts=3):
    """Gauss-Legendre points and weights over x in [0,L], y,z in [-w/2,w/2]."""
    x, wx = np.polynomial.legendre.leggauss(npts)
    px = 0.5 * L * (x + 1.0)
    wpx = 0.5 * L * wx
    py = 0.5 * w * x
    wpy = 0.5 * w * wx
    P = np.array([[a, b, c] for a in px for b in py for c in py])
    W = np.array([wa * wb * wc for wa in wpx for wb in wpy for wc in wpy])
    return P, W


def dof_subtree_links(desc):
    """For every DOF, the boolean mask of links whose pose depends on it."""
    mask = np.zeros((desc.n_dofs, desc.n_links), dtype=bool)
    dof_start = desc.link_dof_start
    for i in range(desc.n_models):
        lo, hi = desc.link_offset[i], desc.link_offset[i + 1]
        for l in range(lo, hi):
            chain = []
            a = l
            while a >= 0:
                chain.append(a)
                par = desc.parent[a]
                a = lo + par if par >= 0 else -1
            for anc in chain:
                for k in range(desc.dofs_per_link[anc]):
                    mask[dof_start[anc] + k, l] = True
    return mask


def pose_jacobian(desc, q):
    """dA_l/dq_n (3x4) for all links and DOFs from the world-frame closed form."""
    T, w, p = link_frames(desc, q)
    mask = dof_subtree_links(desc)
    J = np.zeros((desc.n_dofs, desc.n_links, 3, 4))
    for n in range(desc.n_dofs):
        W = np.array([[0, -w[n, 2], w[n, 1]], [w[n, 2], 0, -w[n, 0]], [-w[n, 1], w[n, 0], 0]])
        for l in np.nonzero(mask[n])[0]:
            J[n, l, :, :3] = W @ T[l, :3, :3]
            J[n, l, :, 3] = np.cross(w[n], T[l, :3, 3] - p[n])
    return J


def full_moment(desc):
    idx = [0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9]
    return desc.mass_moment[:, idx].reshape(-1, 4, 4)


def inertia_matrix(desc, q, model=0):
    J = pose_jacobian(desc, q)
    M = full_moment(desc)
    do = desc.dof_offset
    sl = slice(do[model], do[model + 1])
    Jm = J[sl]
    return np.einsum("ilrx,lxy,jlry->ij", Jm, M, Jm)


# ------------------------------------------------------ Lagrangian reference
def lagrangian_accel(desc, q, qd, h=1e-6):
    """q'' of the continuous equations (Eq. DYN_EXP form): H q'' = -Hdot q' + dT/dq - dV/dq,
    single model, with H and V from the world-frame Jacobian and the FD derivatives of H."""
    g = desc.gravity

    def Hm(qq):
        return inertia_matrix(desc, qq, 0)

    def V(qq):
        T, _, _ = link_frames(desc, qq)
        M = full_moment(desc)
        return -sum(g @ (T[l, :3, :] @ M[l][:, 3]) for l in range(desc.n_links))

    n = desc.n_dofs
    H = Hm(q)
    Hdot = np.zeros((n, n))
    dT = np.zeros(n)
    dV = np.zeros(n)
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        Hp, Hn = Hm(q + e), Hm(q - e)
        dH = (Hp - Hn) / (2 * h)
        Hdot += dH * qd[j]
        dT[j] = 0.5 * qd @ dH @ qd
        dV[j] = (V(q + e) - V(q - e)) / (2 * h)
    return np.linalg.solve(H, -Hdot @ qd + dT - dV)


def rk4_reference(desc, q0, T_end, dt):
    q, v = np.array(q0, dtype=float), np.zeros_like(q0, dtype=float)
    for _ in range(int(round(T_end / dt))):
        k1q, k1v = v, lagrangian_accel(desc, q, v)
        k2q, k2v = v + 0.5 * dt * k1v, lagrangian_accel(desc, q + 0.5 * dt * k1q, v + 0.5 * dt * k1v)
        k3q, k3v = v + 0.5 * dt * k2v, lagrangian_accel(desc, q + 0.5 * dt * k2q, v + 0.5 * dt * k2v)
        k4q, k4v = v + dt * k3v, lagrangian_accel(desc, q + dt * k3q, v + dt * k3v)
        q = q + dt / 6 * (k1q + 2 * k2q + 2 * k3q + k4q)
        v = v + dt / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return q
