"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test checks the oracle against something it does not itself define: the
closed-form semi-implicit Euler solution, textbook pendulum frequencies, energy and
momentum behaviour of a symplectic integrator, the mass matrix and bias rebuilt
from finite differences of the kinematics and of the Lagrangian, static contact
equilibria, Coulomb sliding, the exact linearisation of the discrete map, and
central finite differences of the window loss.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as D
from oracle.dynamics import F64, OracleModel
from oracle.window import mlp_forward, obs_fn, oracle_window, oracle_window_grads, reward_fn

torch.set_num_threads(4)


def T(x):
    return torch.as_tensor(np.asarray(x), dtype=F64)


def run_substeps(m, q, qd, a, dt, n):
    for _ in range(n):
        q, qd = D.substep(m, q, qd, a, dt)
    return q, qd


# ------------------------------------------------------------------ integrator, gravity

def test_free_fall_closed_form():
    """Semi-implicit Euler free fall: z_n = z0 + n dt v0 - g dt^2 n (n+1) / 2."""
    m = OracleModel(wl.free_body())
    q = T([[0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0]])
    qd = torch.zeros(1, 6, dtype=F64)
    dt, n = 1.0 / 240.0, 128
    q, qd = run_substeps(m, q, qd, torch.zeros(1, 0, dtype=F64), dt, n)
    z_ref = 1.0 - 9.81 * dt * dt * n * (n + 1) / 2.0
    assert abs(z_ref - (-0.40610)) < 1e-5
    assert abs(float(q[0, 2]) - z_ref) <= 1e-12 * abs(z_ref)
    assert abs(float(qd[0, 2]) + 9.81 * dt * n) < 1e-12


def _period(theta, dt):
    """Mean period from upward zero crossings with linear interpolation."""
    th = np.asarray(theta)
    idx = np.where((th[:-1] < 0) & (th[1:] >= 0))[0]
    tc = (idx + (-th[idx]) / (th[idx + 1] - th[idx])) * dt
    return (tc[-1] - tc[0]) / (len(tc) - 1), len(tc)


def test_pendulum_period_locked_cart():
    """Rod on a hinge: T = 2 pi sqrt(2L / 3g); discrete T_d = 2 pi dt / acos(1 - w^2 dt^2 / 2)."""
    m = OracleModel(wl.pendulum(mass=0.1, length=1.0))
    dt = 1.0 / 240.0
    w2 = 3.0 * 9.81 / 2.0
    assert abs(2 * np.pi / np.sqrt(w2) - 1.637947) < 1e-6
    Td = 2 * np.pi * dt / np.arccos(1 - w2 * dt * dt / 2)
    assert abs(Td - 1.637929) < 1e-6
    q, qd = T([[1e-4]]), T([[0.0]])
    a = torch.zeros(1, 1, dtype=F64)
    th = []
    for _ in range(int(12 * 1.64 / dt)):
        q, qd = D.substep(m, q, qd, a, dt)
        th.append(float(q[0, 0]))
    Tm, nc = _period(th, dt)
    assert nc >= 10
    assert abs(Tm - Td) / Td < 1e-6


def test_pendulum_period_free_cart():
    """CartPole hanging (angle pi): w^2 = m g l / (I_c + m l^2 - m^2 l^2 / (M + m))."""
    m = OracleModel(wl.cartpole())
    dt = 1.0 / 240.0
    M_, mp, l, Ic = 1.0, 0.1, 0.5, 0.1 / 12
    w2 = mp * 9.81 * l / (Ic + mp * l * l - mp * mp * l * l / (M_ + mp))
    assert abs(2 * np.pi / np.sqrt(w2) - 1.581122) < 1e-6
    Td = 2 * np.pi * dt / np.arccos(1 - w2 * dt * dt / 2)
    assert abs(Td - 1.581104) < 1e-6
    q, qd = T([[0.0, np.pi + 1e-4]]), T([[0.0, 0.0]])
    a = torch.zeros(1, 1, dtype=F64)
    th = []
    for _ in range(int(12 * 1.6 / dt)):
        q, qd = D.substep(m, q, qd, a, dt)
        th.append(float(q[0, 1]) - np.pi)
    Tm, nc = _period(th, dt)
    assert nc >= 10
    assert abs(Tm - Td) / Td < 1e-6


# ------------------------------------------------------------------ energy, momentum

def _energy_error(md, q0, qd0, dt, t_end):
    m = OracleModel(md)
    q, qd = T(q0), T(qd0)
    a = torch.zeros(q.shape[0], m.na, dtype=F64)
    e0 = float(D.kinetic_energy(m, q, qd)[0] + D.potential_energy(m, q))
    err = 0.0
    for _ in range(int(round(t_end / dt))):
        q, qd = D.substep(m, q, qd, a, dt)
        e = float(D.kinetic_energy(m, q, qd)[0] + D.potential_energy(m, q))
        err = max(err, abs(e - e0) / abs(e0))
    return err


def test_energy_error_is_first_order_cartpole():
    md = wl.cartpole()
    q0, qd0 = [[0.0, 2.0]], [[0.3, -0.5]]
    e1 = _energy_error(md, q0, qd0, 1.0 / 120, 5.0)
    e2 = _energy_error(md, q0, qd0, 1.0 / 240, 5.0)
    assert e1 < 0.1
    assert 1.6 < e1 / e2 < 2.4


def test_energy_error_is_first_order_floating_chain_zero_g():
    md = wl.chain(n=4, free_root=True, gravity=0.0)
    m = OracleModel(md)
    rng = np.random.default_rng(3)
    q0 = np.zeros((1, m.nq))
    q0[0, 3] = 1.0
    q0[0, 7:] = rng.normal(size=m.nq - 7) * 0.3
    qd0 = rng.normal(size=(1, m.nv))
    e1 = _energy_error(md, q0, qd0, 1.0 / 400, 1.0)
    e2 = _energy_error(md, q0, qd0, 1.0 / 800, 1.0)
    assert e1 < 0.05
    assert 1.6 < e1 / e2 < 2.4


def _momentum(m, q, qd):
    """Total spatial momentum about the world origin from body COM velocities (FK finite differences free)."""
    T_ = D.dynamics_terms(m, q, qd)
    h = torch.zeros(q.shape[0], 6, dtype=F64)
    for i, j in enumerate(T_["bodies"]):
        h = h + (T_["I6"][:, i] @ T_["V"][j][..., None])[..., 0]
    return h


def test_momentum_drift_in_flight_is_first_order():
    md = wl.chain(n=4, free_root=True, gravity=0.0)
    m = OracleModel(md)
    rng = np.random.default_rng(5)
    q0 = np.zeros((1, m.nq))
    q0[0, 3] = 1.0
    q0[0, 7:] = rng.normal(size=m.nq - 7) * 0.3
    qd0 = rng.normal(size=(1, m.nv))
    a = T(rng.normal(size=(1, m.na)))

    def drift(dt, t_end=0.5):
        q, qd = T(q0), T(qd0)
        h0 = _momentum(m, q, qd)
        worst = 0.0
        for _ in range(int(round(t_end / dt))):
            q, qd = D.substep(m, q, qd, a, dt)
            worst = max(worst, float((_momentum(m, q, qd) - h0).abs().max()))
        return worst, float(h0.abs().max())

    d1, scale = drift(1.0 / 400)
    d2, _ = drift(1.0 / 800)
    assert d1 / scale < 0.3
    assert 1.6 < d1 / d2 < 2.4


# ------------------------------------------------------------------ M and bias in other forms

def _fd_point_and_rotation(m, q, dq, eps):
    """Central differences of every body's COM and rotation along the velocity dq."""
    def advance(qv, s):
        out = qv.clone()
        for j in range(m.J):
            a, v = m.qadr[j], m.vadr[j]
            if m.jtype[j] == D.FREE:
                out[:, a:a + 3] = qv[:, a:a + 3] + s * dq[:, v:v + 3]
                out[:, a + 3:a + 7] = D.quat_exp_update(qv[:, a + 3:a + 7], dq[:, v + 3:v + 6], s)
            else:
                out[:, a] = qv[:, a] + s * dq[:, v]
        return out
    Rp, pp = D.forward_kinematics(m, advance(q, eps))
    Rm, pm = D.forward_kinematics(m, advance(q, -eps))
    R0, _ = D.forward_kinematics(m, q)
    res = {}
    for j in m.bodies:
        cp = pp[j] + Rp[j] @ m.com[j]
        cm = pm[j] + Rm[j] @ m.com[j]
        vc = (cp - cm) / (2 * eps)
        W = (Rp[j] - Rm[j]) / (2 * eps) @ R0[j].transpose(-1, -2)
        w = torch.stack([W[:, 2, 1], W[:, 0, 2], W[:, 1, 0]], -1)
        res[j] = (vc, w, R0[j])
    return res


@pytest.mark.parametrize("name", ["chain_free", "chain_fixed", "ant", "humanoid"])
def test_mass_matrix_from_kinematics(name):
    md = {"chain_free": lambda: wl.chain(4, True), "chain_fixed": lambda: wl.chain(4, False),
          "ant": wl.ant, "humanoid": wl.humanoid}[name]()
    m = OracleModel(md)
    rng = np.random.default_rng(11)
    s0 = wl.initial_states(md, 1, seed=2) if md["task"] != "none" else None
    q = T(s0[:, :m.nq]) if s0 is not None else T(rng.normal(size=(1, m.nq)) * 0.5)
    if m.jtype[0] == D.FREE:
        q[:, 3:7] = T(rng.normal(size=(1, 4)))
        q[:, 3:7] /= q[:, 3:7].norm()
    T_ = D.dynamics_terms(m, q, torch.zeros(1, m.nv, dtype=F64))
    M = T_["M"][0]
    assert torch.allclose(M, M.T, atol=1e-12)
    assert float(torch.linalg.eigvalsh(M).min()) > 0
    # M = sum_b m J_c^T J_c + J_w^T I_w J_w with Jacobian columns from FK differences
    cols = []
    for k in range(m.nv):
        e = torch.zeros(1, m.nv, dtype=F64)
        e[0, k] = 1.0
        cols.append(_fd_point_and_rotation(m, q, e, 1e-6))
    Mfd = torch.diag(m.armature).clone()
    for j in m.bodies:
        Jc = torch.stack([cols[k][j][0][0] for k in range(m.nv)], 1)
        Jw = torch.stack([cols[k][j][1][0] for k in range(m.nv)], 1)
        R0 = cols[0][j][2][0]
        Iw = R0 @ m.inertia[j] @ R0.T
        Mfd = Mfd + m.mass[j] * Jc.T @ Jc + Jw.T @ Iw @ Jw
    assert torch.allclose(M, Mfd, atol=1e-7 * float(M.abs().max()))
    # kinetic energy identity for a random velocity
    qd = T(rng.normal(size=(1, m.nv)))
    ke, _ = D.kinetic_energy(m, q, qd)
    fd = _fd_point_and_rotation(m, q, qd, 1e-6)
    ke_fd = 0.5 * float((qd[0] * T(m.armature) * qd[0]).sum())
    for j in m.bodies:
        vc, w, R0 = fd[j]
        Iw = R0[0] @ m.inertia[j] @ R0[0].T
        ke_fd += 0.5 * float(m.mass[j] * (vc[0] ** 2).sum() + w[0] @ Iw @ w[0])
    assert abs(float(ke[0]) - ke_fd) < 1e-7 * abs(ke_fd)


def test_bias_from_lagrangian_fixed_base():
    """b = Mdot qd - d/dq (qd^T M qd / 2) + dV/dq, all by central differences."""
    md = wl.chain(5, free_root=False, seed=13)
    m = OracleModel(md)
    rng = np.random.default_rng(4)
    q = T(rng.normal(size=(1, m.nq)) * 0.7)
    qd = T(rng.normal(size=(1, m.nv)))
    b = D.dynamics_terms(m, q, qd)["bias"][0]
    eps = 1e-5

    def Mof(qq):
        return D.dynamics_terms(m, qq, torch.zeros_like(qd))["M"][0]

    Mdot_qd = (Mof(q + eps * qd) - Mof(q - eps * qd)) / (2 * eps) @ qd[0]
    grad_T = torch.zeros(m.nv, dtype=F64)
    grad_V = torch.zeros(m.nv, dtype=F64)
    for k in range(m.nv):
        e = torch.zeros_like(q)
        e[0, k] = eps
        grad_T[k] = 0.5 * (qd[0] @ (Mof(q + e) - Mof(q - e)) @ qd[0]) / (2 * eps)
        grad_V[k] = (D.potential_energy(m, q + e) - D.potential_energy(m, q - e))[0] / (2 * eps)
    b_lag = Mdot_qd - grad_T + grad_V
    assert torch.allclose(b, b_lag, atol=1e-7 * float(b_lag.abs().max()) + 1e-9)


def test_free_body_com_acceleration_and_euler_equations():
    """Torque-free body with offset COM: COM accelerates at g; I w' + w x I w = 0."""
    md = wl.free_body(mass=2.0, inertia=(0.1, 0.2, 0.3))
    md["com"][0] = np.array([0.1, -0.2, 0.05])
    m = OracleModel(md)
    rng = np.random.default_rng(9)
    qu = rng.normal(size=4)
    q = T(np.concatenate([[0.3, 0.1, 1.0], qu / np.linalg.norm(qu)])[None])
    qd = T(rng.normal(size=(1, 6)))
    T_ = D.dynamics_terms(m, q, qd)
    qdd = torch.linalg.solve(T_["M"], (-T_["bias"])[..., None])[..., 0][0]
    R = T_["R"][0][0]
    c_rel = R @ m.com[0]
    w, vp = qd[0, 3:], qd[0, :3]
    ap, alpha = qdd[:3], qdd[3:]
    a_com = ap + torch.linalg.cross(alpha, c_rel) + torch.linalg.cross(w, torch.linalg.cross(w, c_rel))
    assert torch.allclose(a_com, T([0, 0, -9.81]), atol=1e-10)
    Iw = R @ m.inertia[0] @ R.T
    assert torch.allclose(Iw @ alpha + torch.linalg.cross(w, Iw @ w), torch.zeros(3, dtype=F64),
                          atol=1e-10)


def test_solve_matches_numpy():
    W = wl.workload("humanoid", 2)
    m = OracleModel(W["model"])
    s = T(W["s0"])
    q, qd = s[:, :m.nq], T(np.random.default_rng(1).normal(size=(2, m.nv)))
    T_ = D.dynamics_terms(m, q, qd)
    rhs = np.random.default_rng(2).normal(size=(2, m.nv))
    L = torch.linalg.cholesky(T_["M"])
    x = torch.cholesky_solve(T(rhs)[..., None], L)[..., 0].numpy()
    for i in range(2):
        x_np = np.linalg.solve(T_["M"][i].numpy(), rhs[i])
        assert np.allclose(x[i], x_np, rtol=1e-12, atol=1e-12)
        assert np.allclose(L[i].numpy(), np.linalg.cholesky(T_["M"][i].numpy()), atol=1e-12)


# ------------------------------------------------------------------ contact

def test_sphere_rests_at_static_penetration():
    md = wl.free_body(mass=2.0, inertia=(0.1, 0.1, 0.1), radius=0.1, contact=True,
                      kn=4e4, kd=1e4, kt=1e3, mu=0.75)
    m = OracleModel(md)
    q = T([[0.0, 0.0, 0.1, 1.0, 0.0, 0.0, 0.0]])
    qd = torch.zeros(1, 6, dtype=F64)
    q, qd = run_substeps(m, q, qd, torch.zeros(1, 0, dtype=F64), 1.0 / 2000, 20000)
    d = float(q[0, 2]) - 0.1
    assert abs(d - (-2.0 * 9.81 / 4e4)) < 1e-5 * 2.0 * 9.81 / 4e4


def test_block_normal_forces_sum_to_weight():
    md = wl.sliding_block(mass=1.5, radius=0.05, kn=4e4, kd=1e4, kt=1e3, mu=0.75)
    m = OracleModel(md)
    q = T([[0.0, 0.0, 0.05, 1.0, 0.0, 0.0, 0.0]])
    qd = torch.zeros(1, 6, dtype=F64)
    q, qd = run_substeps(m, q, qd, torch.zeros(1, 0, dtype=F64), 1.0 / 2000, 20000)
    T_ = D.dynamics_terms(m, q, qd)
    fz = float(T_["contact_f"][0, :, 2].sum())
    assert abs(fz - 1.5 * 9.81) < 1e-5 * 1.5 * 9.81


def test_coulomb_sliding_decelerates_at_mu_g():
    """All contacts in the Coulomb branch: friction totals mu * sum|f_n| = mu m g."""
    mass, mu, kn = 1.0, 0.75, 4e4
    md = wl.sliding_block(mass=mass, radius=0.05, kn=kn, kd=1e4, kt=1e3, mu=mu)
    m = OracleModel(md)
    d_eq = -mass * 9.81 / (4 * kn)
    q = T([[0.0, 0.0, 0.05 + d_eq, 1.0, 0.0, 0.0, 0.0]])
    qd = T([[1.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    dt, n = 1.0 / 4000, 400
    T_ = D.dynamics_terms(m, q, qd)
    assert float(T_["contact_f"][0, :, 2].sum()) == pytest.approx(mass * 9.81, rel=1e-9)
    q, qd = run_substeps(m, q, qd, torch.zeros(1, 0, dtype=F64), dt, n)
    decel = (1.0 - float(qd[0, 0])) / (n * dt)
    assert decel == pytest.approx(mu * 9.81, rel=2e-3)


def test_viscous_friction_decays_at_kt_over_m():
    mass, kt = 2.0, 1e3
    md = wl.free_body(mass=mass, inertia=(100.0, 100.0, 100.0), radius=0.1, contact=True,
                      kn=4e4, kd=1e4, kt=kt, mu=0.75)
    m = OracleModel(md)
    d_eq = -mass * 9.81 / 4e4
    v0 = 1e-4
    q = T([[0.0, 0.0, 0.1 + d_eq, 1.0, 0.0, 0.0, 0.0]])
    qd = T([[v0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    dt, n = 1e-4, 20
    T_ = D.dynamics_terms(m, q, qd)
    assert kt * v0 < 0.75 * abs(float(T_["contact_f"][0, 0, 2]))
    q, qd = run_substeps(m, q, qd, torch.zeros(1, 0, dtype=F64), dt, n)
    assert float(qd[0, 0]) / v0 == pytest.approx((1 - kt * dt / mass) ** n, rel=1e-3)


def test_contact_force_law_values():
    """Single sphere: hand-evaluated normal force and both friction branches."""
    md = wl.free_body(mass=1.0, radius=0.1, contact=True, kn=4e4, kd=1e4, kt=1e3, mu=0.75)
    m = OracleModel(md)
    q = T([[0.0, 0.0, 0.099, 1.0, 0.0, 0.0, 0.0]])        # d = -1e-3
    for vx, branch in ((1e-3, "viscous"), (1.0, "coulomb")):
        qd = T([[vx, 0.0, -0.2, 0.0, 0.0, 0.0]])
        f = D.dynamics_terms(m, q, qd)["contact_f"][0, 0]
        fn = (-4e4 + 1e4 * -0.2) * -1e-3
        assert float(f[2]) == pytest.approx(fn, rel=1e-12)
        ft = -1e3 * vx if branch == "viscous" else -0.75 * fn
        assert float(f[0]) == pytest.approx(ft, rel=1e-12)
    qd = T([[1.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    q_air = T([[0.0, 0.0, 0.2, 1.0, 0.0, 0.0, 0.0]])
    assert float(D.dynamics_terms(m, q_air, qd)["contact_f"].abs().max()) == 0.0


def test_joint_limit_penalty_values():
    md = wl.ant()
    m = OracleModel(md)
    q = torch.zeros(1, m.nq, dtype=F64)
    q[0, 3] = 1.0
    j = 2                                             # first knee, limits 30..70 deg
    q[0, m.qadr[j]] = np.deg2rad(20)
    tau = D.joint_torques(m, q, torch.zeros(1, m.na, dtype=F64))[0]
    assert float(tau[m.vadr[j]]) == pytest.approx(1e4 * np.deg2rad(10), rel=1e-12)
    q[0, m.qadr[j]] = np.deg2rad(80)
    tau = D.joint_torques(m, q, torch.zeros(1, m.na, dtype=F64))[0]
    assert float(tau[m.vadr[j]]) == pytest.approx(-1e4 * np.deg2rad(10), rel=1e-12)
    q[0, m.qadr[j]] = np.deg2rad(50)
    tau = D.joint_torques(m, q, torch.ones(1, m.na, dtype=F64))[0]
    assert float(tau[m.vadr[j]]) == pytest.approx(50.0, rel=1e-12)


# ------------------------------------------------------------------ rewards, obs, MLP

def test_humanoid_standing_reward_and_obs():
    W = wl.workload("humanoid", 1)
    m = OracleModel(W["model"])
    s = torch.zeros(1, 76, dtype=F64)
    s[0, 2] = 1.348
    s[0, 3] = 1.0
    a = torch.zeros(1, 21, dtype=F64)
    # v = 0, up = heading = 1, height term 10 * clip(1.348 - 0.84, -1, 0.1) = 1
    assert float(reward_fn(m, s, a)[0]) == pytest.approx(0.1 + 1.0 + 1.0, abs=1e-14)
    a[0, :] = 0.5
    s[0, 2] = 0.74
    assert float(reward_fn(m, s, a)[0]) == pytest.approx(0.1 + 1.0 - 200 * 0.01 - 0.002 * 21 * 0.25)
    o = obs_fn(m, s)
    assert o.shape == (1, 76)
    assert float(o[0, 53]) == 1.0 and float(o[0, 54]) == 1.0


def test_cartpole_reward_wraps_angle():
    m = OracleModel(wl.cartpole())
    s = T([[0.5, 2 * np.pi + 0.1, 0.2, -0.3]])
    r = float(reward_fn(m, s, torch.zeros(1, 1, dtype=F64))[0])
    assert r == pytest.approx(-0.01 - 0.1 * 0.09 - 0.05 * 0.25 - 0.1 * 0.04, abs=1e-12)


def test_mlp_elu_tanh_small_case():
    W1, b1 = T([[1.0, -2.0], [0.5, 0.5]]), T([0.0, -1.0])
    W2, b2 = T([[1.0, 1.0]]), T([0.25])
    y = mlp_forward([(W1, b1), (W2, b2)], T([[1.0, 1.0]]))
    # hidden: [-1 -> e^-1 - 1, 0 -> 0] ; out = e^-1 - 1 + 0 + 0.25
    assert float(y[0, 0]) == pytest.approx(np.exp(-1) - 1 + 0.25, abs=1e-15)


# ------------------------------------------------------------------ exact linearisation

@pytest.mark.parametrize("upright", [False, True])
def test_linearisation_is_matrix_power(upright):
    """At an equilibrium with zero action, d s_n / d s_0 = Phi^n of the linear scheme."""
    m = OracleModel(wl.pendulum())
    dt, n = 1.0 / 240, 200
    w2 = 3.0 * 9.81 / 2.0 * (-1.0 if upright else 1.0)
    Phi = np.array([[1 - dt * dt * w2, dt], [-dt * w2, 1.0]])
    th0 = np.pi if upright else 0.0

    def f(x):
        q, qd = x[:, :1], x[:, 1:]
        q, qd = run_substeps(m, q, qd, torch.zeros(1, 1, dtype=F64), dt, n)
        return torch.cat([q, qd], 1)

    J = torch.autograd.functional.jacobian(f, T([[th0, 0.0]]))[0, :, 0, :].numpy()
    P = np.linalg.matrix_power(Phi, n)
    assert np.allclose(J, P, rtol=1e-10, atol=1e-10 * np.abs(P).max())


def test_linearisation_free_cart_blocks():
    m = OracleModel(wl.cartpole())
    dt, n = 1.0 / 240, 100
    T_ = D.dynamics_terms(m, T([[0.0, np.pi]]), torch.zeros(1, 2, dtype=F64))
    M = T_["M"][0].numpy()
    # gravity torque m g l sin(theta) linearises to -m g l (theta - pi): qdd = -M^{-1} K q
    A = np.linalg.solve(M, np.diag([0.0, 0.1 * 9.81 * 0.5]))
    I2 = np.eye(2)
    Phi = np.block([[I2 - dt * dt * A, dt * I2], [-dt * A, I2]])

    def f(x):
        q, qd = x[:, :2], x[:, 2:]
        q, qd = run_substeps(m, q, qd, torch.zeros(1, 1, dtype=F64), dt, n)
        return torch.cat([q, qd], 1)

    J = torch.autograd.functional.jacobian(f, T([[0.0, np.pi, 0.0, 0.0]]))[0, :, 0, :].numpy()
    P = np.linalg.matrix_power(Phi, n)
    assert np.allclose(J, P, rtol=1e-9, atol=1e-9 * np.abs(P).max())


# ------------------------------------------------------------------ window adjoint vs FD

def _fd_check(W, h, envs, coords_a, coords_s, eps, tol, closed_loop=True):
    md = W["model"]
    s0 = W["s0"][envs]
    N = W["n_envs"]
    actor = W["actor"] if closed_loop else None
    acts = None
    if not closed_loop:
        rng = np.random.default_rng(7)
        acts = np.tanh(rng.normal(size=(h, len(envs), md["na"])))
    g = oracle_window_grads(md, s0, h, actor, W["critic"], actions=acts, n_total=N)
    m = OracleModel(md)
    lay = ([(T(Wt), T(b)) for Wt, b in W["actor"]], [(T(Wt), T(b)) for Wt, b in W["critic"]])

    def loss(ds=None, da=None):
        s = T(s0).clone()
        if ds is not None:
            s = s + T(ds)
        return float(oracle_window(m, s, h, actions=acts, n_total=N, layers=lay,
                                   action_offset=da)["loss"])
    L0 = abs(loss())
    floor = 50 * 2.2e-16 * L0 / eps        # roundoff of a central difference of L
    worst = 0.0
    for (t, e, k) in coords_a:
        da = np.zeros((h, len(envs), md["na"]))
        da[t, e, k] = eps
        fd = (loss(da=da) - loss(da=-da)) / (2 * eps)
        an = g["dL_da"][t, e, k]
        worst = max(worst, abs(fd - an) / (abs(fd) + 1e-12 * (1 + abs(an))))
        assert abs(fd - an) <= tol * abs(fd) + floor, (t, e, k, fd, an)
    for (e, k) in coords_s:
        ds = np.zeros_like(s0)
        ds[e, k] = eps
        fd = (loss(ds=ds) - loss(ds=-ds)) / (2 * eps)
        an = g["dL_ds0"][e, k]
        assert abs(fd - an) <= tol * abs(fd) + floor, (e, k, fd, an)
    return worst


def test_window_adjoint_fd_cartpole_every_coordinate():
    W = wl.workload("cartpole")
    h = 32
    envs = [0, 5]
    coords_a = [(t, e, 0) for t in range(h) for e in range(len(envs))]
    coords_s = [(e, k) for e in range(len(envs)) for k in range(4)]
    _fd_check(W, h, envs, coords_a, coords_s, 1e-6, 1e-6)


def test_window_adjoint_fd_ant_short():
    W = wl.workload("ant", 64)
    h = 2
    rng = np.random.default_rng(0)
    coords_a = [(t, 0, int(k)) for t in range(h) for k in rng.choice(8, 3, replace=False)]
    coords_s = [(0, int(k)) for k in rng.choice(37, 8, replace=False)]
    _fd_check(W, h, [3], coords_a, coords_s, 1e-6, 1e-5)


def test_policy_weight_fd_like_paper_check():
    """FD of the loss along single actor weights vs the reverse-mode dL/dtheta (App. A.5)."""
    W = wl.workload("cartpole")
    h = 16
    s0 = W["s0"][:4]
    g = oracle_window_grads(W["model"], s0, h, W["actor"], W["critic"], n_total=16,
                            want_theta=True)
    for (li, idx) in ((0, (3, 1)), (1, (10, 20)), (2, (0, 5))):
        eps = 1e-6
        Wp = [(x.copy(), y.copy()) for x, y in W["actor"]]
        Wm = [(x.copy(), y.copy()) for x, y in W["actor"]]
        Wp[li][0][idx] += eps
        Wm[li][0][idx] -= eps
        lp = float(oracle_window(W["model"], s0, h, Wp, W["critic"], n_total=16)["loss"])
        lm = float(oracle_window(W["model"], s0, h, Wm, W["critic"], n_total=16)["loss"])
        fd = (lp - lm) / (2 * eps)
        an = g["dL_dtheta"][li][0][idx]
        floor = 50 * 2.2e-16 * abs(lp) / eps
        assert abs(fd - an) <= 1e-6 * abs(fd) + floor, (li, idx, fd, an)


def test_window_adjoint_fd_open_loop_ant():
    W = wl.workload("ant", 64)
    h = 2
    coords_a = [(0, 0, 1), (1, 0, 6), (0, 0, 3)]
    coords_s = [(0, 2), (0, 20), (0, 33)]
    _fd_check(W, h, [11], coords_a, coords_s, 1e-6, 1e-5, closed_loop=False)


# ------------------------------------------------------------------ the paper's printed constants

def _golden():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_reward_coefficients_match_the_paper():
    G = _golden()
    m = OracleModel(wl.cartpole())
    c = G["cartpole_reward"]
    base = T([[0.0, 0.0, 0.0, 0.0]])
    for idx, key in ((1, "theta2"), (3, "thetadot2"), (0, "x2"), (2, "xdot2")):
        s = base.clone()
        s[0, idx] = 0.5
        assert float(reward_fn(m, s, torch.zeros(1, 1, dtype=F64))[0]) == pytest.approx(c[key] * 0.25)
    for name in ("ant", "humanoid"):
        W = wl.workload(name, 1)
        m = OracleModel(W["model"])
        g = G[f"{name}_reward"]
        ns = W["s0"].shape[1]
        s = torch.zeros(1, ns, dtype=F64)
        s[0, 3] = 1.0
        a = torch.zeros(1, m.na, dtype=F64)
        if name == "ant":
            s[0, 2] = 1.0
            r0 = float(reward_fn(m, s, a)[0])
            assert r0 == pytest.approx(g["up"] + g["heading"] + 1.0 - g["height_offset"])
        else:
            s[0, 2] = g["height_target"] + 0.05
            r0 = float(reward_fn(m, s, a)[0])
            assert r0 == pytest.approx(g["up"] + g["heading"] + g["above"] * 0.05)
            s2 = s.clone()
            s2[0, 2] = g["height_target"] - 0.3
            assert float(reward_fn(m, s2, a)[0]) == pytest.approx(g["up"] + g["heading"] + g["below"] * 0.09)
            s3 = s.clone()
            s3[0, 2] = g["height_target"] + 5.0
            assert float(reward_fn(m, s3, a)[0]) == pytest.approx(g["up"] + g["heading"] + g["above"] * g["clip_hi"])
            a2 = torch.full((1, m.na), 0.5, dtype=F64)
            assert float(reward_fn(m, s, a2)[0]) == pytest.approx(r0 + g["action"] * 0.25 * m.na)
        s4 = s.clone()
        s4[0, m.nq] = 0.7
        assert float(reward_fn(m, s4, a)[0]) == pytest.approx(r0 + g["vx"] * 0.7)


def test_obs_and_action_dimensions_match_the_paper():
    G = _golden()
    for name in ("cartpole", "ant", "humanoid"):
        W = wl.workload(name, 2)
        m = OracleModel(W["model"])
        o = obs_fn(m, T(W["s0"]))
        assert o.shape[1] == G["obs_dims"][name]
        assert m.na == G["action_dims"][name]


def test_discounted_loss_closed_form():
    """CartPole hanging at rest with zero actions and a constant critic c0:
    L = pi^2 (1 - g^h) / ((1 - g) h) - g^h c0 / h."""
    G = _golden()
    gamma, h = G["gamma"]["value"], G["horizon"]["value"]
    md = wl.cartpole()
    N = 3
    s0 = np.tile([[0.0, np.pi, 0.0, 0.0]], (N, 1))
    c0 = 0.37
    critic = [(np.zeros((4, 5)), np.zeros(4)), (np.zeros((1, 4)), np.array([c0]))]
    acts = np.zeros((h, N, 1))
    out = oracle_window(md, s0, h, None, critic, actions=acts, gamma=gamma)
    ref = np.pi ** 2 * (1 - gamma ** h) / ((1 - gamma) * h) - gamma ** h * c0 / h
    assert float(out["loss"]) == pytest.approx(ref, rel=1e-12)


# ------------------------------------------------------------------ muscle-tendon units

def _arm_state(md, theta, x=0.1, xd=0.0, thd=0.0, act=0.5):
    return T([[x, theta, xd, thd, act]])


@pytest.mark.parametrize("via", [None, 0.45])
def test_muscle_path_length_rate_and_torque_closed_form(via):
    """Cart + pole with one muscle (origin on the cart, insertion on the pole, optionally a
    via point on the pole): L(theta) = sqrt(b^2+d^2-2bd sin th) [+ via form], the cart force
    vanishes (the tension is internal to the chain) and the hinge torque is -F dL/dtheta."""
    d, b = 0.3, 0.8
    md = wl.muscle_arm(d=d, b=b, c=via)
    m = OracleModel(md)
    for th, thd in ((0.3, 1.7), (-0.8, -0.4), (1.2, 0.9)):
        s = _arm_state(md, th, thd=thd)
        q, qd, act = s[:, :2], s[:, 2:4], s[:, 4:5]
        Tm = D.dynamics_terms(m, q, qd)
        mt = D.muscle_terms(m, Tm, qd, act)
        if via is None:
            L = np.sqrt(b * b + d * d - 2 * b * d * np.sin(th))
            dL = -b * d * np.cos(th) / L
        else:
            c = via
            Lc = np.sqrt(c * c + d * d - 2 * c * d * np.sin(th))
            L = Lc + (b - c)
            dL = -c * d * np.cos(th) / Lc
        assert float(mt["L"][0, 0]) == pytest.approx(L, rel=1e-13)
        assert float(mt["Ldot"][0, 0]) == pytest.approx(dL * thd, rel=1e-12)
        F = float(mt["F"][0, 0])
        assert F > 0
        tau = mt["tau"][0].numpy()
        assert abs(tau[0]) < 1e-12 * F
        assert tau[1] == pytest.approx(-F * dL, rel=1e-12)


def test_muscle_force_length_velocity_special_cases():
    """At l_m = l_opt and zero lengthening rate the tension is F_max * act; it falls to
    F_max act exp(-1) one width away, and vanishes at the maximum shortening speed."""
    d, b = 0.3, 0.8
    th = 0.4
    L = np.sqrt(b * b + d * d - 2 * b * d * np.sin(th))
    lslack = 0.2
    for lt, fl in ((1.0, 1.0), (1.45, np.exp(-1.0)), (0.55, np.exp(-1.0))):
        lopt = (L - lslack) / lt
        md = wl.muscle_arm(d=d, b=b, fmax=80.0, lopt=lopt, lslack=lslack)
        m = OracleModel(md)
        s = _arm_state(md, th, act=0.25)
        Tm = D.dynamics_terms(m, s[:, :2], s[:, 2:4])
        F = float(D.muscle_terms(m, Tm, s[:, 2:4], s[:, 4:5])["F"][0, 0])
        assert F == pytest.approx(80.0 * 0.25 * fl, rel=1e-12)
    # shortening at v_max * l_opt: f_v = 0
    lopt = L - lslack
    md = wl.muscle_arm(d=d, b=b, lopt=lopt, lslack=lslack)
    m = OracleModel(md)
    dL = -b * d * np.cos(th) / L
    thd = -10.0 * lopt / dL        # Ldot = -v_max l_opt
    s = _arm_state(md, th, thd=thd)
    Tm = D.dynamics_terms(m, s[:, :2], s[:, 2:4])
    mt = D.muscle_terms(m, Tm, s[:, 2:4], s[:, 4:5])
    assert abs(float(mt["F"][0, 0])) < 1e-9


def test_muscle_power_balance_humanoid():
    """For the 152-unit humanoid at a random state: the power of the generalized muscle
    forces equals minus the sum of tension times lengthening rate (virtual work), and the
    lengthening rate equals the central difference of the path length along qd."""
    md = wl.mtu_humanoid()
    m = OracleModel(md)
    W = wl.workload("mtu", 3)
    rng = np.random.default_rng(11)
    s = T(W["s0"])
    nq, nv = m.nq, m.nv
    q = s[:, :nq]
    qd = T(rng.normal(0.0, 0.5, (3, nv)))
    act = T(rng.uniform(0.1, 0.9, (3, m.n_mtu)))
    Tm = D.dynamics_terms(m, q, qd)
    mt = D.muscle_terms(m, Tm, qd, act)
    power = (mt["tau"] * qd).sum(1)
    assert torch.allclose(power, -(mt["F"] * mt["Ldot"]).sum(1), rtol=1e-12, atol=1e-9)
    eps = 1e-6
    qp = D.integrate(m, q, qd, eps)
    qm = D.integrate(m, q, qd, -eps)
    Lp = D.muscle_terms(m, D.dynamics_terms(m, qp, qd), qd, act)["L"]
    Lm = D.muscle_terms(m, D.dynamics_terms(m, qm, qd), qd, act)["L"]
    fd = (Lp - Lm) / (2 * eps)
    assert torch.allclose(fd, mt["Ldot"], rtol=1e-6, atol=1e-8)


def test_activation_lag_closed_form():
    """Explicit activation recursion with constant excitation u:
    a_n = u + (a_0 - u) (1 - dt/tau)^n."""
    md = wl.muscle_arm()
    m = OracleModel(md)
    dt = 1.0 / 240.0
    a = T([[0.1]])
    u = T([[0.8]])
    for n in range(1, 40):
        a = D.activation_step(m, a, u, dt)
        want = 0.8 + (0.1 - 0.8) * (1.0 - dt / m.tau_act) ** n
        assert float(a[0, 0]) == pytest.approx(want, rel=1e-13)


def test_muscle_arm_window_adjoint_fd():
    """Open-loop excitations on the muscle arm over 6 frames: every dL/du_t and dL/ds0
    coordinate against central differences."""
    md = wl.muscle_arm()
    m = OracleModel(md)
    h = 6
    rng = np.random.default_rng(3)
    s0 = np.array([[0.05, 0.3, 0.2, -0.5, 0.3], [0.0, -0.6, 0.0, 0.4, 0.7]])
    u = rng.uniform(0.1, 0.9, (h, 2, 1))
    critic = [(rng.normal(size=(1, 5)), np.zeros(1))]      # linear value of the observed state
    g = oracle_window_grads(md, s0, h, None, critic, actions=u, n_total=2)
    lay = (None, [(T(Wc), T(bc)) for Wc, bc in critic])

    def loss(ds=None, du=None):
        s = T(s0) + (T(ds) if ds is not None else 0.0)
        return float(oracle_window(m, s, h, actions=u, n_total=2, action_offset=du, layers=lay)["loss"])
    eps = 1e-6
    for t in range(h):
        for e in range(2):
            du = np.zeros_like(u)
            du[t, e, 0] = eps
            fd = (loss(du=du) - loss(du=-du)) / (2 * eps)
            assert fd == pytest.approx(g["dL_da"][t, e, 0], rel=1e-6, abs=1e-11)
    for e in range(2):
        for k in range(5):
            ds = np.zeros_like(s0)
            ds[e, k] = eps
            fd = (loss(ds=ds) - loss(ds=-ds)) / (2 * eps)
            assert fd == pytest.approx(g["dL_ds0"][e, k], rel=1e-6, abs=1e-11)


def test_mtu_reward_coefficients_match_the_paper():
    G = _golden()["mtu_reward"]
    W = wl.workload("mtu", 1)
    m = OracleModel(W["model"])
    s = torch.zeros(1, W["s0"].shape[1], dtype=F64)
    s[0, 3] = 1.0
    a = torch.zeros(1, m.na, dtype=F64)
    s[0, 2] = 0.84 + 0.02
    r0 = float(reward_fn(m, s, a)[0])
    assert r0 == pytest.approx(G["up"] + G["heading"] + G["above"] * 0.02)
    s2 = s.clone()
    s2[0, 2] = 0.84 + 3.0
    assert float(reward_fn(m, s2, a)[0]) == pytest.approx(G["up"] + G["heading"] + G["above"] * G["clip_hi"])
    s3 = s.clone()
    s3[0, 2] = 0.84 - 0.3
    assert float(reward_fn(m, s3, a)[0]) == pytest.approx(G["up"] + G["heading"] + G["below"] * 0.09)
    a2 = torch.full((1, m.na), 0.5, dtype=F64)
    assert float(reward_fn(m, s, a2)[0]) == pytest.approx(r0 + G["action"] * 0.25 * m.na)
    assert m.n_mtu == _golden()["mtu_dims"]["muscles"] and m.na == _golden()["mtu_dims"]["actions"]


def test_mtu_observation_layout_and_squash():
    """Skeleton entries as in the humanoid observation (without the last action), zeros up
    to entry 128, then the activations; excitations are (tanh + 1)/2 in (0, 1)."""
    from oracle import squash
    Wm = wl.workload("mtu", 2)
    Wh = wl.workload("humanoid", 2)
    m = OracleModel(Wm["model"])
    mh = OracleModel(Wh["model"])
    s = T(Wm["s0"]).clone()
    s[:, 55:] = T(np.linspace(0.0, 1.0, 152))[None]
    o = obs_fn(m, s)
    sh = torch.cat([s[:, :55], torch.zeros(2, 21, dtype=F64)], 1)
    oh = obs_fn(mh, sh)
    assert o.shape == (2, 280)
    assert torch.equal(o[:, :55], oh[:, :55])
    assert torch.equal(o[:, 55:128], torch.zeros(2, 73, dtype=F64))
    assert torch.equal(o[:, 128:], s[:, 55:])
    y = T([[-30.0, 0.0, 30.0]])
    u = squash(m, y)
    assert float(u[0, 1]) == 0.5 and 0.0 <= float(u[0, 0]) < 1e-12 and 1 - 1e-12 < float(u[0, 2]) <= 1.0


def test_bf16_rounding_matches_library_conversion_and_ties():
    """bf16_round agrees with torch's float32 -> bfloat16 conversion (round to nearest
    even) on random values, keeps bfloat16 values, and sends exact ties to the even
    neighbour."""
    from oracle import bf16_round
    x = torch.randn(20000, dtype=F64) * 10.0 ** torch.randint(-6, 6, (20000,)).to(F64)
    want = x.to(torch.float32).to(torch.bfloat16).to(F64)
    assert torch.equal(bf16_round(x), want)
    exact = want
    assert torch.equal(bf16_round(exact), exact)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert float(bf16_round(T([1.0 + 2.0 ** -8]))[0]) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert float(bf16_round(T([1.0 + 3 * 2.0 ** -8]))[0]) == 1.0 + 2.0 ** -6


def test_bf16_linear_backward_is_rounded_transpose_product():
    """The BF16 MLP's reverse: input adjoint bf16(dy) bf16(W), weight adjoint
    dy^T bf16(x), checked on one layer against the explicit products."""
    from oracle import bf16_round, mlp_forward_bf16
    rng = np.random.default_rng(5)
    W = T(rng.normal(size=(7, 5)))
    b = T(rng.normal(size=7))
    x = T(rng.normal(size=(3, 5))).requires_grad_(True)
    Wg = W.clone().requires_grad_(True)
    y = mlp_forward_bf16([(Wg, b)], x)
    gy = T(rng.normal(size=(3, 7)))
    y.backward(gy)
    assert torch.equal(y.detach(), bf16_round(x.detach()) @ bf16_round(W).T + b)
    assert torch.equal(x.grad, bf16_round(gy) @ bf16_round(W))
    assert torch.allclose(Wg.grad, gy.T @ bf16_round(x.detach()), rtol=1e-15, atol=0)


def test_stochastic_policy_zero_sigma_and_log_std_gradient():
    """Stochastic policy of the oracle (reparameterised sample mu + exp(log_std) eps):
    sigma -> 0 gives the deterministic window, and dL/dlog_std from reverse mode agrees
    with central differences of the loss in log_std."""
    import workloads as wl
    from oracle import oracle_window, oracle_window_grads
    W = wl.workload("cartpole", 4)
    h = 6
    rng = np.random.default_rng(21)
    eps = rng.standard_normal((h, 4, 1))
    det = oracle_window(W["model"], W["s0"], h, W["actor"], W["critic"])
    zero = oracle_window(W["model"], W["s0"], h, W["actor"], W["critic"], noise=eps,
                         log_std=np.array([-np.inf]))
    assert float(det["loss"]) == float(zero["loss"])
    ls = np.array([-0.7])
    g = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], want_theta=True,
                            noise=eps, log_std=ls)
    e = 1e-6
    lp = float(oracle_window(W["model"], W["s0"], h, W["actor"], W["critic"], noise=eps, log_std=ls + e)["loss"])
    lm = float(oracle_window(W["model"], W["s0"], h, W["actor"], W["critic"], noise=eps, log_std=ls - e)["loss"])
    fd = (lp - lm) / (2 * e)
    assert abs(g["dL_dlog_std"][0] - fd) <= 1e-6 * max(1.0, abs(fd))
    assert abs(fd) > 1e-8


def test_early_termination_restarts_window():
    """Early termination in the oracle: an env that falls below the termination height in
    frame 0 continues exactly as a fresh window from its reset state (its later rewards
    discounted from the reset), and nothing flows back through the reset into s_0."""
    import workloads as wl
    from oracle import oracle_window, oracle_window_grads
    W = wl.workload("ant", 1)
    md = wl.with_termination(W["model"])
    s_low = W["s0"].copy()
    s_low[:, 2] = 0.2                                   # root below 0.27 m
    reset = wl.initial_states(md, 1, seed=9)
    h = 4
    A = oracle_window(md, s_low, h, W["actor"], None, reset_states=reset)
    assert A["done"][:, 0].tolist() == [True, False, False, False]
    B = oracle_window(md, reset, h - 1, W["actor"], None)
    r0 = float(A["rewards"][0][0])
    assert abs(4 * float(A["loss"]) - 3 * float(B["loss"]) + r0) < 1e-12
    gA = oracle_window_grads(md, s_low, h, W["actor"], None, reset_states=reset)
    g1 = oracle_window_grads(md, s_low, 1, W["actor"], None)      # loss -r_0 alone
    np.testing.assert_allclose(gA["dL_ds0"], g1["dL_ds0"] / 4, rtol=0, atol=1e-14)
    # with no env below the height the window is the one without termination
    C = oracle_window(md, W["s0"], h, W["actor"], W["critic"], reset_states=reset)
    D = oracle_window(W["model"], W["s0"], h, W["actor"], W["critic"])
    assert not C["done"].any() and float(C["loss"]) == float(D["loss"])


def test_observation_normalisation_is_a_first_layer_fold():
    """Observation normalisation (Sec. 3.3) in the oracle: reading (o - mu) * s through a first
    layer (W, b) is the layer (W diag(s), b - W (mu * s)) on raw o, so the normalised window
    equals the raw window with folded actor and critic (loss, dL/da, dL/ds0), and the actor's
    first-layer gradients map back by dL/dW = dL/dW' diag(s) - dL/db' (mu * s)^T, dL/db = dL/db'."""
    import workloads as wl
    from oracle import oracle_window_grads
    W = wl.workload("ant", 3)
    od = W["obs_dim"]
    rng = np.random.default_rng(4)
    mu = rng.normal(0.0, 0.5, od)
    sc = rng.uniform(0.3, 2.0, od)

    def fold(layers):
        (W0, b0), rest = layers[0], layers[1:]
        return [(W0 * sc[None, :], b0 - W0 @ (mu * sc))] + list(rest)
    h = 3
    A = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], want_theta=True, obs_norm=(mu, sc))
    B = oracle_window_grads(W["model"], W["s0"], h, fold(W["actor"]), fold(W["critic"]), want_theta=True)
    assert abs(A["loss"] - B["loss"]) < 1e-12 * abs(B["loss"])
    for key in ("actions", "rewards", "value", "dL_da", "dL_ds0", "obs"):
        np.testing.assert_allclose(A[key], B[key], rtol=1e-9, atol=1e-12)
    (gW, gb), (fW, fb) = A["dL_dtheta"][0], B["dL_dtheta"][0]
    np.testing.assert_allclose(gb, fb, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(gW, fW * sc[None, :] - np.outer(fb, mu * sc), rtol=1e-8, atol=1e-13)
    for (a1, a2), (b1, b2) in zip(A["dL_dtheta"][1:], B["dL_dtheta"][1:]):
        np.testing.assert_allclose(a1, b1, rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(a2, b2, rtol=1e-9, atol=1e-14)


def test_adhesive_contact_count_threshold():
    """The literal normal force (-k_n + k_d d_dot) min(d, 0) of Sec. 3.1 pulls exactly when a
    penetrating contact separates faster than k_n / k_d: an Ant lowered 5 cm (its 4 foot
    spheres penetrate), moving straight up at k_n / k_d +- 0.5 m/s, counts all penetrating
    contacts or none as pulling in its first substep."""
    import workloads as wl
    from oracle import OracleModel, substep, dynamics_terms
    W = wl.workload("ant", 1)
    m = OracleModel(W["model"])
    s0 = torch.as_tensor(W["s0"], dtype=torch.float64)
    q, qd = s0[:, :m.nq].clone(), torch.zeros(1, m.nv, dtype=torch.float64)
    q[:, 2] -= 0.05
    a = torch.zeros(1, m.na, dtype=torch.float64)
    vcrit = m.kn / m.kd
    npen = int((dynamics_terms(m, q, qd)["contact_d"] < 0.0).sum())
    assert npen == 4
    for vz, want in ((vcrit + 0.5, npen), (vcrit - 0.5, 0), (-1.0, 0)):
        qd[:, 2] = vz
        stats = []
        substep(m, q, qd, a, m.dt / m.substeps, stats=stats)
        assert int(stats[0][0]) == want, (vz, int(stats[0][0]))


# ------------------------------------------------------------------ observation tables, value by value

def _obs_tables():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "obs_tables.json")))


def _blocks(rows):
    """Start index and width of every row of an observation table."""
    out, i = {}, 0
    for name, n in rows:
        out[name] = (i, n)
        i += n
    return out, i


def test_cartpole_obs_entries_follow_the_table():
    """Every entry of the CartPole observation on a hand-built state, in the order and with
    the widths of App. A.3's table: x, x_dot, (sin theta, cos theta), theta_dot."""
    blk, n = _blocks(_obs_tables()["cartpole"]["rows"])
    m = OracleModel(wl.cartpole())
    x, th, xd, thd = 0.3, 2.0, -0.7, 1.9
    o = obs_fn(m, T([[x, th, xd, thd]]))[0].numpy()
    assert o.shape == (n,)
    want = {"cart_position": [x], "cart_velocity": [xd], "sin_cos_pole_angle": [np.sin(th), np.cos(th)],
            "pole_angular_velocity": [thd]}
    for name, (i, w) in blk.items():
        assert np.array_equal(o[i:i + w], np.asarray(want[name])), name


@pytest.mark.parametrize("name", ["ant", "humanoid"])
def test_floating_base_obs_entries_follow_the_table(name):
    """Every entry of the Ant / Humanoid observation on a hand-built state with distinct
    values, block by block as App. A.3's table lists them.  The root is turned by
    Rz(alpha) Rx(beta), so the up projection (body z on world z) is cos(beta) and the heading
    projection (body x on world x) is cos(alpha), in closed form."""
    tab = _obs_tables()[name]
    blk, n = _blocks(tab["rows"])
    W = wl.workload(name, 1)
    md = W["model"]
    m = OracleModel(md)
    nq, nv, na = m.nq, m.nv, m.na
    nh = nq - 7
    alpha, beta = 0.7, 0.4
    ca, sa, cb, sb = np.cos(alpha / 2), np.sin(alpha / 2), np.cos(beta / 2), np.sin(beta / 2)
    quat = [ca * cb, ca * sb, sa * sb, sa * cb]
    pos = [1.5, -2.5, 0.9]
    hinge = 0.01 * (np.arange(nh) + 1)
    vlin, vang = [0.11, 0.22, 0.33], [-0.44, 0.55, -0.66]
    hvel = -0.1 * (np.arange(nh) + 1)
    aprev = 0.5 - 0.03 * np.arange(na)
    s = np.concatenate([pos, quat, hinge, vlin, vang, hvel, aprev])[None]
    o = obs_fn(m, T(s))[0].numpy()
    assert o.shape == (n,)
    want = {"base_height": [pos[2]], "torso_height": [pos[2]],
            "base_quaternion": quat, "torso_quaternion": quat,
            "base_linear_velocity": vlin, "torso_linear_velocity": vlin,
            "base_angular_velocity": vang, "torso_angular_velocity": vang,
            "joint_angles": hinge, "joint_velocities": hvel,
            "up_heading": [np.cos(beta), np.cos(alpha)], "last_actions": aprev}
    for row, (i, w) in blk.items():
        np.testing.assert_allclose(o[i:i + w], np.asarray(want[row]), rtol=0, atol=1e-15, err_msg=row)


# ------------------------------------------------------------------ humanoid window adjoint vs FD, 8 envs

def test_window_adjoint_fd_humanoid_eight_envs_every_coordinate():
    """Central differences (eps 1e-6) of each env's loss term over a 4-frame humanoid window
    (App. A.5's finite-difference check), on the 8 envs of the headline batch drawn with seed 4:
    every action coordinate of every frame and every initial-state coordinate except the root
    quaternion, against the reverse-mode dL/da and dL/ds0.  The envs are independent, so all
    the perturbed windows run as one batch of copies and each copy's own loss term is read.
    The window is piecewise smooth (a contact switches on at the first substep it penetrates),
    so a pair whose +-eps interval holds such a switch is not differentiable there; those pairs
    (at most 1 % of them) are differenced again at eps / 10, where the switch falls outside."""
    W = wl.workload("humanoid", 1024)
    md, N, h, eps = W["model"], 1024, 4, 1e-6
    envs = np.sort(np.random.default_rng(4).choice(N, 8, replace=False))
    s0 = W["s0"][envs]
    E, ns, na = len(envs), s0.shape[1], md["na"]
    g = oracle_window_grads(md, s0, h, W["actor"], W["critic"], n_total=N)
    coords = [("a", t, k) for t in range(h) for k in range(na)] + [("s", k) for k in range(ns) if not 3 <= k < 7]
    m = OracleModel(md)
    lay = ([(T(Wt), T(b)) for Wt, b in W["actor"]], [(T(Wt), T(b)) for Wt, b in W["critic"]])

    def central(pairs, step):
        """Central differences of the env's loss term for (coordinate index, env index) pairs."""
        S0 = np.repeat(s0[[e for _, e in pairs]], 2, 0)
        DA = np.zeros((h, 2 * len(pairs), na))
        for i, (c, _) in enumerate(pairs):
            co = coords[c]
            for sg, sign in enumerate((1.0, -1.0)):
                if co[0] == "a":
                    DA[co[1], 2 * i + sg, co[2]] = sign * step
                else:
                    S0[2 * i + sg, co[1]] += sign * step
        le = []
        chunk = 512
        for i in range(0, S0.shape[0], chunk):
            out = oracle_window(m, T(S0[i:i + chunk]), h, n_total=N, layers=lay,
                                action_offset=DA[:, i:i + chunk], diagnostics=False)
            le.append(out["loss_env"].numpy())
        le = np.concatenate(le).reshape(len(pairs), 2)
        return (le[:, 0] - le[:, 1]) / (2 * step)

    pairs = [(c, e) for c in range(len(coords)) for e in range(E)]
    an = np.array([g["dL_da"][coords[c][1], e, coords[c][2]] if coords[c][0] == "a" else g["dL_ds0"][e, coords[c][1]]
                   for c, e in pairs])
    L0 = np.abs(oracle_window(m, T(s0), h, n_total=N, layers=lay, diagnostics=False)["loss_env"].numpy())
    L0p = np.array([L0[e] for _, e in pairs])
    fd = central(pairs, eps)
    bad = np.abs(fd - an) > 1e-5 * np.abs(fd) + 50 * 2.2e-16 * L0p / eps
    assert bad.mean() <= 0.01, bad.sum()
    redo = [p for p, b in zip(pairs, bad) if b]
    if redo:
        fd2 = central(redo, eps / 10)
        an2, L2 = an[bad], L0p[bad]
        still = np.abs(fd2 - an2) > 1e-5 * np.abs(fd2) + 50 * 2.2e-16 * L2 / (eps / 10)
        assert not still.any(), [(coords[c], int(envs[e]), f, a) for (c, e), f, a, s in zip(redo, fd2, an2, still) if s]
    assert np.abs(an).max() > 0 and (np.abs(an) > 0).mean() > 0.9


# ------------------------------------------------------------------ recursive form vs defining form

@pytest.mark.parametrize("name", ["cartpole", "ant", "humanoid"])
def test_recursive_algorithms_equal_the_defining_form(name):
    """The composite-rigid-body mass matrix and the recursive Newton-Euler inverse dynamics
    equal the defining sums over bodies (M = sum J^T I J, b = sum J^T (I (Jdot qd - a_g) +
    V x* I V), contacts through point Jacobians) on random states with penetrating contacts,
    and a recursive substep equals the oracle's substep, to rounding."""
    from oracle import recursive as RC
    W = wl.workload(name, 4)
    m = OracleModel(W["model"])
    rng = np.random.default_rng(11)
    q = T(W["s0"])[:, :m.nq].clone()
    if name != "cartpole":
        q[:, 7:] += T(rng.normal(0, 0.3, (4, m.nq - 7)))
        q[:, 2] -= 0.05                                  # push the contact spheres into the ground
    qd = T(rng.normal(size=(4, m.nv)))
    qdd = T(rng.normal(size=(4, m.nv)))
    a = T(rng.uniform(-1, 1, (4, m.na)))
    Td = D.dynamics_terms(m, q, qd)
    if name != "cartpole":
        assert bool((Td["contact_d"] < 0).any())
    M = RC.mass_matrix(m, q)
    assert float((M - Td["M"]).abs().max()) <= 1e-13 * float(Td["M"].abs().max())
    b = Td["bias"] - Td["tau_contact"]
    ID0 = RC.inverse_dynamics(m, q, qd, torch.zeros_like(qd))
    assert float((ID0 - b).abs().max()) <= 1e-13 * float(b.abs().max())
    ID1 = RC.inverse_dynamics(m, q, qd, qdd)
    want = ID0 + (Td["M"] @ qdd[..., None])[..., 0]
    assert float((ID1 - want).abs().max()) <= 1e-13 * float(want.abs().max())
    q1, qd1 = D.substep(m, q, qd, a, 1.0 / 240)
    q2, qd2, _, _ = RC.substep_recursive(m, q, qd, a, 1.0 / 240)
    assert float((q1 - q2).abs().max()) <= 1e-12 and float((qd1 - qd2).abs().max()) <= 1e-12 * float(qd1.abs().max())


# ------------------------------------------------------------------ the FP32 storage floor mode

def test_fp32_floor_mode_off_is_the_fp64_window_and_on_stores_float32():
    """Off, the floor switch changes nothing (bitwise).  On, every state after a frame,
    every action and the initial state hold float32 values (the storage an FP32 simulator
    has) while the arithmetic stays FP64, the result moves by about the float32 resolution,
    and the gradients are the FP64 adjoint along the rounded trajectory (straight through the
    rounding): on a one-frame CartPole window they agree with the plain FP64 gradients to the
    size of that move."""
    from oracle.window import fp32_round
    W = wl.workload("cartpole")
    md, h = W["model"], 3
    a = oracle_window(md, W["s0"], h, W["actor"], W["critic"])
    b = oracle_window(md, W["s0"], h, W["actor"], W["critic"], fp32_floor=False)
    for key in ("value", "loss", "loss_env"):
        assert torch.equal(a[key], b[key])
    for x, y in zip(a["states"], b["states"]):
        assert torch.equal(x, y)
    c = oracle_window(md, W["s0"], h, W["actor"], W["critic"], fp32_floor=True)
    for x in c["states"] + c["actions"]:
        assert torch.equal(x, x.to(torch.float32).to(F64))
    d = float((c["states"][-1] - a["states"][-1]).abs().max() / a["states"][-1].abs().max())
    assert 1e-9 < d < 1e-5
    x = T([1.0 + 2.0 ** -30, 3.0]).requires_grad_(True)
    y = fp32_round(x)
    assert float(y[0].detach()) == 1.0 and float(y[1].detach()) == 3.0
    g, = torch.autograd.grad((y * T([2.0, 5.0])).sum(), x)
    assert torch.equal(g, T([2.0, 5.0]))
    r0 = oracle_window_grads(md, W["s0"], 1, W["actor"], W["critic"])
    r1 = oracle_window_grads(md, W["s0"], 1, W["actor"], W["critic"], fp32_floor=True)
    for key in ("dL_da", "dL_ds0"):
        assert np.linalg.norm(r1[key] - r0[key]) <= 1e-5 * np.linalg.norm(r0[key])
    assert np.abs(r1["loss_env"].sum() - r1["loss"]) <= 1e-15 * abs(r1["loss"])


def test_fp32_floor_file_is_the_oracles_and_states_the_conditioning():
    """tests/golden/fp32_floor.json holds the oracle's own numbers: its one-frame humanoid row
    is recomputed here, and its summary follows from its rows.  It also states the
    conditioning of the headline window: at h = 32 no sampled env's FP32 storage floor is under
    the parity bar (an FP32 window cannot meet it there), while at h = 1 every one is."""
    import json
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_fp32_floor as MF
    with open(os.path.join(os.path.dirname(__file__), "golden", "fp32_floor.json")) as fh:
        fl = json.load(fh)
    hum = fl["humanoid"]
    assert hum["envs"] == [int(e) for e in np.sort(np.random.default_rng(4).choice(1024, 8, replace=False))]
    row = MF.floor_rows("humanoid", 1024, hum["envs"], [1])[0]
    stored = next(r for r in hum["rows"] if r["h"] == 1)
    for a, b in zip(row["per_env"], stored["per_env"]):
        for key in ("dL_da_rel", "dL_ds0_rel", "s_h_rel"):
            assert a[key] == pytest.approx(b[key], rel=1e-9, abs=1e-18), key
    summary = MF.summarise(json.loads(json.dumps(fl)))
    for key in ("humanoid", "mtu"):
        assert summary[key]["h_max_under_bar"] == fl[key]["h_max_under_bar"]
        assert summary[key]["h_gate"] == fl[key]["h_gate"] <= fl[key]["h_max_under_bar"]
    r32 = next(r for r in hum["rows"] if r["h"] == 32)
    assert not any(MF.under_bar(e) for e in r32["per_env"])
    assert all(MF.under_bar(e) for e in next(r for r in hum["rows"] if r["h"] == 1)["per_env"])


# ------------------------------------------------------------------ layer normalisation of the hidden layers

def test_layer_norm_hand_case_and_library():
    """The oracle's layer normalisation on a hand-computed row (mean 2, population variance
    2/3) and against torch's own layer_norm on random rows; the MLP applies it after each
    hidden layer's ELU and not after the output layer."""
    from oracle.window import layer_norm
    a = T([[1.0, 2.0, 3.0]])
    g, b = T([2.0, 1.0, 0.5]), T([0.1, 0.0, -0.1])
    s = np.sqrt(2.0 / 3.0 + 1e-5)
    want = [2.0 * (-1.0 / s) + 0.1, 0.0, 0.5 * (1.0 / s) - 0.1]
    assert np.allclose(layer_norm(a, g, b, 1e-5)[0].numpy(), want, rtol=0, atol=1e-15)
    x = T(np.random.default_rng(1).normal(size=(5, 7)))
    g7, b7 = T(np.linspace(0.5, 1.5, 7)), T(np.linspace(-0.2, 0.2, 7))
    lib = torch.nn.functional.layer_norm(x, (7,), g7, b7, 1e-5)
    assert torch.allclose(layer_norm(x, g7, b7, 1e-5), lib, rtol=0, atol=1e-14)
    W1, b1 = T([[1.0, -2.0], [0.5, 0.5], [2.0, 1.0]]), T([0.0, -1.0, 0.3])
    W2, b2 = T([[1.0, 1.0, -1.0]]), T([0.25])
    x2 = T([[1.0, 1.0]])
    gl, bl = T([1.0, 2.0, 0.5]), T([0.0, 0.1, 0.2])
    hid = torch.nn.functional.elu(x2 @ W1.T + b1)
    want_y = layer_norm(hid, gl, bl, 1e-5) @ W2.T + b2
    assert torch.allclose(mlp_forward([(W1, b1), (W2, b2)], x2, [(gl, bl)]), want_y, rtol=0, atol=1e-15)


def test_window_adjoint_fd_with_layer_norm_cartpole():
    """Central differences of the CartPole window loss with layer normalisation on the actor's
    and critic's hidden layers: every action and initial-state coordinate of two envs over 8
    frames, and single gains / biases of the actor's normalisations against dL/dln."""
    W = wl.workload("cartpole")
    md, h, N, eps = W["model"], 8, 16, 1e-6
    rng = np.random.default_rng(2)
    aln = [(rng.uniform(0.5, 1.5, 64), rng.normal(0, 0.1, 64)) for _ in range(2)]
    cln = [(rng.uniform(0.5, 1.5, 64), rng.normal(0, 0.1, 64)) for _ in range(2)]
    s0 = W["s0"][[0, 5]]
    g = oracle_window_grads(md, s0, h, W["actor"], W["critic"], n_total=N, want_theta=True, actor_ln=aln,
                            critic_ln=cln)
    m = OracleModel(md)
    lay = ([(T(Wt), T(b)) for Wt, b in W["actor"]], [(T(Wt), T(b)) for Wt, b in W["critic"]])

    def loss(ds=None, da=None, ln=aln):
        s = T(s0).clone() + (T(ds) if ds is not None else 0.0)
        return float(oracle_window(m, s, h, n_total=N, layers=lay, action_offset=da, actor_ln=ln,
                                   critic_ln=cln)["loss"])
    L0 = abs(loss())
    floor = 50 * 2.2e-16 * L0 / eps
    for t in range(h):
        for e in range(2):
            da = np.zeros((h, 2, 1))
            da[t, e, 0] = eps
            fd = (loss(da=da) - loss(da=-da)) / (2 * eps)
            assert abs(fd - g["dL_da"][t, e, 0]) <= 1e-6 * abs(fd) + floor, (t, e)
    for e in range(2):
        for k in range(4):
            ds = np.zeros_like(s0)
            ds[e, k] = eps
            fd = (loss(ds=ds) - loss(ds=-ds)) / (2 * eps)
            assert abs(fd - g["dL_ds0"][e, k]) <= 1e-6 * abs(fd) + floor, (e, k)
    for (li, which, j) in ((0, 0, 3), (1, 1, 40), (1, 0, 7)):
        lp = [(x.copy(), y.copy()) for x, y in aln]
        lm = [(x.copy(), y.copy()) for x, y in aln]
        lp[li][which][j] += eps
        lm[li][which][j] -= eps
        fd = (loss(ln=lp) - loss(ln=lm)) / (2 * eps)
        an = g["dL_dln"][li][which][j]
        assert abs(fd - an) <= 1e-6 * abs(fd) + floor, (li, which, j, fd, an)
