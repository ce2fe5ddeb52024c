"""The recursive form of the substep dynamics, in FP64 (TEST INFRASTRUCTURE ONLY).

The oracle's own substep (``dynamics.substep``) builds the mass matrix and the bias in
their defining dense form.  This module states the same equations of motion (Sec. 3.1, Eq.
"fwd_dynamics", with the readings of ``dynamics``) through the recursive algorithms that
Sec. 3.1 names for an articulated simulator:

* forward kinematics and the spatial velocities and bias accelerations of every frame by a
  pass from the root outwards (the velocity of a frame is its parent's plus its own joint's
  motion S q_dot);
* inverse dynamics by the recursive Newton-Euler algorithm: the Newton-Euler force of every
  body, minus the external contact wrench, is accumulated from the leaves inwards and
  projected on each joint's motion subspace, giving ID(q, q_dot, q_ddot) = M q_ddot + b - J^T f;
* the mass matrix by the composite-rigid-body algorithm: composite inertias accumulated from
  the leaves inwards, M[i][j] = S_i^T (I^c_j S_j) for every frame i on the root path of j;
* q_ddot = M^{-1}(tau - ID(q, q_dot, 0)) by a Cholesky factorisation, then the same
  semi-implicit Euler step.

It serves two purposes: the pins of the test suite hold it equal to the defining form to
rounding (so the two formulations check each other), and the operation counter counts it
(``count_ops.count_recursive_substep``) to give the algorithmic operation count of one substep
and of its adjoint by the implicit-function theorem (lambda = M^{-1} q_ddot_bar by the two
triangular solves of the factor, then the vector-Jacobian product of ID at the solved
q_ddot), which the benchmark's roofline uses.  Torque-driven models only.
"""
import torch

from .dynamics import F64, FREE, cross, fcross, forward_kinematics, integrate, joint_torques, mcross, \
    motion_subspace, skew


def _spatial_inertia(m, R, p, j):
    """World-frame spatial inertia [B, 6, 6] of body j about the origin (mass, centre of mass,
    rotational inertia about the centre of mass turned into world axes)."""
    c = p[j] + R[j] @ m.com[j]
    Ic = R[j] @ m.inertia[j] @ R[j].transpose(-1, -2)
    C = skew(c)
    mass = m.mass[j]
    eye = torch.eye(3, dtype=F64).expand(C.shape)
    return torch.cat([torch.cat([Ic + mass * (C @ C.transpose(-1, -2)), mass * C], -1),
                      torch.cat([mass * C.transpose(-1, -2), mass * eye], -1)], -2)


def _mv(A, x):
    return (A @ x[..., None])[..., 0]


def kinematics(m, q, qd):
    """Frame transforms, motion subspaces, spatial inertias of the bodies, spatial velocities
    and each joint's velocity-product acceleration S_dot q_dot, root outwards."""
    B = q.shape[0]
    R, p = forward_kinematics(m, q)
    S = [motion_subspace(m, R, p, j) for j in range(m.J)]
    I = [_spatial_inertia(m, R, p, j) if float(m.mass[j]) > 0.0 else None for j in range(m.J)]
    V, C = [], []
    for j in range(m.J):
        par, a, nd = m.parent[j], m.vadr[j], m.ndof(j)
        u = _mv(S[j], qd[:, a:a + nd])
        vpar = V[par] if par >= 0 else torch.zeros(B, 6, dtype=F64)
        if m.jtype[j] == FREE:
            vp, w = qd[:, a:a + 3], qd[:, a + 3:a + 6]
            c = torch.cat([torch.zeros_like(w), cross(vp, w)], -1)
        else:
            c = mcross(vpar, u)
        V.append(vpar + u)
        C.append(c)
    return dict(R=R, p=p, S=S, I=I, V=V, C=C)


def contact_wrenches(m, R, p, V):
    """Per body, the world wrench (about the origin) of its contact spheres' forces (the
    contact law of ``dynamics``: penalty normal force, linear-step friction, both only while
    the sphere penetrates)."""
    W = {}
    zhat = torch.tensor([0.0, 0.0, 1.0], dtype=F64)
    for c, b in enumerate(m.cbody):
        xc = p[b] + R[b] @ m.cpos[c]
        xp = xc - m.crad[c] * zhat
        v = V[b][:, 3:] + cross(V[b][:, :3], xp)
        d = xc[:, 2] - m.crad[c]
        pen = torch.where(d < 0.0, d, torch.zeros_like(d))
        fn = (-m.kn + m.kd * v[:, 2]) * pen
        vt = torch.cat([v[:, :2], torch.zeros_like(v[:, 2:])], -1)
        vt2 = (vt * vt).sum(-1)
        afn = torch.abs(fn)
        viscous = (m.kt * m.kt * vt2) <= (m.mu * afn) ** 2
        vn = torch.sqrt(torch.where(viscous, torch.ones_like(vt2), vt2))
        ft = torch.where(viscous[:, None], -m.kt * vt, -(m.mu * afn / vn)[:, None] * vt)
        ft = torch.where((d < 0.0)[:, None], ft, torch.zeros_like(ft))
        f = ft + fn[:, None] * zhat
        w = torch.cat([cross(xp, f), f], -1)
        W[b] = W[b] + w if b in W else w
    return W


def inverse_dynamics(m, q, qd, qdd, kin=None, wc=None):
    """Recursive Newton-Euler: the generalized forces M q_ddot + b(q, q_dot) - J_c^T f_c that
    produce q_ddot, with gravity as a base acceleration and the contact wrenches (evaluated at
    q, q_dot) as external forces.  kin / wc: the kinematics of (q, q_dot) and the contact
    wrenches, when already computed."""
    B = q.shape[0]
    k = kin if kin is not None else kinematics(m, q, qd)
    S, V, C, Ib = k["S"], k["V"], k["C"], k["I"]
    g0 = torch.zeros(B, 6, dtype=F64)
    g0[:, 5] = m.g                                   # the base accelerates upward at g
    Wc = wc if wc is not None else contact_wrenches(m, k["R"], k["p"], V)
    A, F = [], []
    for j in range(m.J):
        par, a, nd = m.parent[j], m.vadr[j], m.ndof(j)
        apar = A[par] if par >= 0 else g0
        A.append(apar + _mv(S[j], qdd[:, a:a + nd]) + C[j])
        if Ib[j] is not None:
            f = _mv(Ib[j], A[j]) + fcross(V[j], _mv(Ib[j], V[j]))
        else:
            f = torch.zeros(B, 6, dtype=F64)
        if j in Wc:
            f = f - Wc[j]
        F.append(f)
    tau = [None] * m.J
    for j in range(m.J - 1, -1, -1):
        tau[j] = (S[j].transpose(-1, -2) @ F[j][..., None])[..., 0]
        if m.parent[j] >= 0:
            F[m.parent[j]] = F[m.parent[j]] + F[j]
    return torch.cat(tau, 1) + m.armature * qdd


def mass_matrix(m, q, kin=None):
    """Composite-rigid-body algorithm, plus the armature on the diagonal.  kin: the
    kinematics of q, when already computed."""
    B = q.shape[0]
    k = kin if kin is not None else kinematics(m, q, torch.zeros(B, m.nv, dtype=F64))
    S = k["S"]
    Ic = [I if I is not None else torch.zeros(B, 6, 6, dtype=F64) for I in k["I"]]
    for j in range(m.J - 1, 0, -1):
        if m.parent[j] >= 0:
            Ic[m.parent[j]] = Ic[m.parent[j]] + Ic[j]
    rows = [[None] * m.J for _ in range(m.J)]
    for j in range(m.J):
        Fj = Ic[j] @ S[j]                            # [B, 6, nd_j]
        i = j
        while i >= 0:
            blk = S[i].transpose(-1, -2) @ Fj         # [B, nd_i, nd_j]
            rows[i][j] = blk
            rows[j][i] = blk.transpose(-1, -2)
            i = m.parent[i]
    for i in range(m.J):
        for j in range(m.J):
            if rows[i][j] is None:
                rows[i][j] = torch.zeros(B, m.ndof(i), m.ndof(j), dtype=F64)
    M = torch.cat([torch.cat(r, 2) for r in rows], 1)
    return M + torch.diag(m.armature)


def substep_recursive(m, q, qd, a, dt):
    """One semi-implicit Euler substep with the recursive algorithms; returns (q', qd', qdd,
    L) with L the Cholesky factor of M."""
    kin = kinematics(m, q, qd)
    tau = joint_torques(m, q, a) - inverse_dynamics(m, q, qd, torch.zeros_like(qd), kin=kin)
    L = torch.linalg.cholesky(mass_matrix(m, q, kin=kin))
    qdd = torch.cholesky_solve(tau[..., None], L)[..., 0]
    qd_new = qd + dt * qdd
    return integrate(m, q, qd_new, dt), qd_new, qdd, L
