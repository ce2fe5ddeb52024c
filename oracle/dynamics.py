"""FP64 articulated-body dynamics of one substep (oracle; test infrastructure only).

Conventions (the readings of the paper's Sec. 3.1 that the whole project uses):

* Spatial vectors are 6-vectors in world Plücker coordinates at the world origin:
  motion (w, v_O), force (n_O, f).  z is up, gravity is (0, 0, -g), the ground is
  z = 0 with normal +z.
* The free root has q = (p, quaternion w,x,y,z) and qd = (world velocity of the
  root origin, world angular velocity).  Its rotation matrix is that of the
  normalised quaternion, R = I + 2 w [v]x + 2 [v]x^2.
* c of Eq. "fwd_dynamics" is minus the bias b(q, qd): Coriolis, centrifugal and
  gravity terms.  External contact forces enter as J^T f.
* Mass matrix (defining form):  M = sum_b J_b^T I_b J_b + diag(armature).
* Bias (defining form, Kane / virtual work):
      b = sum_b J_b^T ( I_b (Jdot_b qd - a_g) + V_b x* I_b V_b ),
  where Jdot_b qd is the time derivative of the body Jacobian applied to qd.
* qdd = M^{-1} (tau + J_c^T f_c - b) through a Cholesky factorisation (Sec. 3.1).
* Semi-implicit Euler: qd' = qd + dt qdd, then positions with qd'; the root
  orientation is left-multiplied by the exact exponential of (dt/2) w'.
* Contact (Sec. 3.1, contact equation): a sphere of radius r at point c of body b;
  penetration d = z_centre - r, contact point = lowest point of the sphere,
  f_n = (-k_n + k_d ddot) min(d, 0) with min active only for d < 0;
  friction (only while d < 0) f_t = -k_t v_t when k_t |v_t| <= mu |f_n| (viscous
  branch, ties included), else -mu |f_n| v_t / |v_t|.
* Joint limits (Sec. 3.1, limit equation): k_lim (lo - q) if q < lo, k_lim (hi - q)
  if q > hi, else 0.
* Muscle-tendon units (Sec. 3.1, muscle actuation; the Hill-type reading of this
  project): a polyline path through points fixed in body frames, length L and rate Ldot;
  rigid tendon l_m = L - l_slack; force-length exp(-((l_m/l_opt - 1)/w)^2);
  force-velocity 1 + Ldot/(v_max l_opt); F = max(0, F_max act f_l f_v), pulling every
  path point towards its neighbours (purely contractive); at a raw tension of exactly 0
  (zero activation, the initial state) the derivative is that of the active branch, the
  side a non-negative activation lies on; the activation follows
  act' = act + dt (u - act)/tau with the excitation u, explicit per substep.
"""
import torch

F64 = torch.float64
FREE, HINGE, SLIDE = 0, 1, 2


def _t(x):
    return torch.as_tensor(x, dtype=F64)


def cross(a, b):
    return torch.linalg.cross(a, b, dim=-1)


def skew(v):
    z = torch.zeros_like(v[..., 0])
    return torch.stack([torch.stack([z, -v[..., 2], v[..., 1]], -1),
                        torch.stack([v[..., 2], z, -v[..., 0]], -1),
                        torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def mcross(a, b):
    """Spatial motion cross product a x b."""
    aw, av, bw, bv = a[..., :3], a[..., 3:], b[..., :3], b[..., 3:]
    return torch.cat([cross(aw, bw), cross(aw, bv) + cross(av, bw)], -1)


def fcross(a, f):
    """Spatial force cross product a x* f."""
    aw, av, fn, ff = a[..., :3], a[..., 3:], f[..., :3], f[..., 3:]
    return torch.cat([cross(aw, fn) + cross(av, ff), cross(aw, ff)], -1)


def quat_mul(a, b):
    aw, av, bw, bv = a[..., :1], a[..., 1:], b[..., :1], b[..., 1:]
    return torch.cat([aw * bw - (av * bv).sum(-1, keepdim=True),
                      aw * bv + bw * av + cross(av, bv)], -1)


def quat_to_rot(qu):
    qn = qu / torch.sqrt((qu * qu).sum(-1, keepdim=True))
    w, v = qn[..., 0], qn[..., 1:]
    V = skew(v)
    eye = torch.eye(3, dtype=F64).expand(V.shape)
    return eye + 2.0 * w[..., None, None] * V + 2.0 * (V @ V)


def axis_angle(axis, ang):
    """Rotation by ``ang`` [B] about the fixed unit ``axis`` [3] (Rodrigues)."""
    K = skew(axis)
    eye = torch.eye(3, dtype=F64)
    return eye + torch.sin(ang)[:, None, None] * K + (1.0 - torch.cos(ang))[:, None, None] * (K @ K)


def quat_exp_update(quat, w, dt):
    """exp((dt/2) w) (x) quat, the exact rotation by angle |w| dt about w / |w|."""
    u = (w * w).sum(-1)
    hh = 0.5 * dt
    x2 = u * hh * hh
    small = x2 < 1e-6
    c_tay = 1.0 - x2 / 2.0 + x2 * x2 / 24.0
    s_tay = hh * (1.0 - x2 / 6.0 + x2 * x2 / 120.0)
    us = torch.where(small, torch.ones_like(u), u)
    n = torch.sqrt(us)
    c = torch.where(small, c_tay, torch.cos(n * hh))
    s = torch.where(small, s_tay, torch.sin(n * hh) / n)
    dq = torch.cat([c[..., None], s[..., None] * w], -1)
    return quat_mul(dq, quat)


class OracleModel:
    """Model tables in float64 tensors, read from a workload model description."""

    def __init__(self, md):
        self.md = md
        self.J = int(md["n_joints"])
        self.nq, self.nv, self.na = int(md["nq"]), int(md["nv"]), int(md["na"])
        self.parent = [int(x) for x in md["parent"]]
        self.jtype = [int(x) for x in md["jtype"]]
        self.qadr = [int(x) for x in md["qadr"]]
        self.vadr = [int(x) for x in md["vadr"]]
        self.offset = _t(md["offset"])
        self.axis = _t(md["axis"])
        self.mass = _t(md["mass"])
        self.com = _t(md["com"])
        self.inertia = _t(md["inertia"])
        self.limited = [bool(x) for x in md["limited"]]
        self.lower = _t(md["lower"])
        self.upper = _t(md["upper"])
        self.act_joint = [int(x) for x in md["act_joint"]]
        self.gear = _t(md["gear"])
        self.armature = _t(md["armature"])
        self.cbody = [int(x) for x in md["contact_body"]]
        self.cpos = _t(md["contact_pos"])
        self.crad = _t(md["contact_radius"])
        self.g = float(md["gravity"])
        self.kn, self.kd, self.kt, self.mu = (float(md[k]) for k in ("kn", "kd", "kt", "mu"))
        self.klim = float(md["klim"])
        self.dt = float(md["dt"])
        self.substeps = int(md["substeps"])
        self.bodies = [j for j in range(self.J) if float(md["mass"][j]) > 0.0]
        self.n_mtu = int(md.get("n_mtu", 0))
        self.n_motor = int(md.get("n_motor", self.na))
        if self.n_mtu:
            self.mtu_npt = [int(x) for x in md["mtu_npt"]]
            self.mtu_body = torch.as_tensor(md["mtu_body"], dtype=torch.long)
            self.mtu_pos = _t(md["mtu_pos"])
            self.mtu_fmax = _t(md["mtu_fmax"])
            self.mtu_lopt = _t(md["mtu_lopt"])
            self.mtu_lslack = _t(md["mtu_lslack"])
            self.tau_act = float(md["tau_act"])
            self.fl_width = float(md["fl_width"])
            self.vmax = float(md["vmax"])
            P = self.mtu_pos.shape[1]
            self.mtu_valid = torch.tensor([[k < n for k in range(P)] for n in self.mtu_npt])

    def ndof(self, j):
        return 6 if self.jtype[j] == FREE else 1


def forward_kinematics(m, q):
    """World rotation R_j [B,3,3] and origin p_j [B,3] of every joint frame."""
    R, p = [], []
    B = q.shape[0]
    for j in range(m.J):
        a, par, jt = m.qadr[j], m.parent[j], m.jtype[j]
        if par >= 0:
            Rp, pp = R[par], p[par]
        else:
            Rp = torch.eye(3, dtype=F64).expand(B, 3, 3)
            pp = torch.zeros(B, 3, dtype=F64)
        base = pp + Rp @ m.offset[j]
        if jt == FREE:
            R.append(quat_to_rot(q[:, a + 3:a + 7]))
            p.append(q[:, a:a + 3])
        elif jt == HINGE:
            R.append(Rp @ axis_angle(m.axis[j], q[:, a]))
            p.append(base)
        else:
            R.append(Rp)
            p.append(base + (Rp @ m.axis[j]) * q[:, a:a + 1])
    return R, p


def motion_subspace(m, R, p, j):
    """World-frame motion subspace S_j [B,6,ndof] of joint j."""
    B = R[j].shape[0]
    jt = m.jtype[j]
    if jt == FREE:
        e = torch.eye(3, dtype=F64).expand(B, 3, 3)
        zero = torch.zeros(B, 3, 3, dtype=F64)
        pe = cross(p[j][:, None, :].expand(B, 3, 3), e)          # rows: p x e_k
        lin = torch.cat([zero, e], 1)                            # columns (0, e_k)
        ang = torch.cat([e, pe.transpose(1, 2)], 1)              # columns (e_k, p x e_k)
        return torch.cat([lin, ang], 2)
    s = R[j] @ m.axis[j]
    if jt == HINGE:
        return torch.cat([s, cross(p[j], s)], -1)[:, :, None]
    return torch.cat([torch.zeros_like(s), s], -1)[:, :, None]


def dynamics_terms(m, q, qd):
    """Everything the equations of motion need at (q, qd), in defining form."""
    B = q.shape[0]
    R, p = forward_kinematics(m, q)
    S = [motion_subspace(m, R, p, j) for j in range(m.J)]
    Jb, V, A = [], [], []
    for j in range(m.J):
        par, a, nd = m.parent[j], m.vadr[j], m.ndof(j)
        base = Jb[par] if par >= 0 else torch.zeros(B, 6, m.nv, dtype=F64)
        cols = [base[:, :, :a], base[:, :, a:a + nd] + S[j], base[:, :, a + nd:]]
        Jj = torch.cat(cols, 2)
        Jb.append(Jj)
        qdj = qd[:, a:a + nd]
        V.append((Jj @ qd[:, :, None])[..., 0])
        if m.jtype[j] == FREE:
            vp, w = qd[:, a:a + 3], qd[:, a + 3:a + 6]
            Sdot_qd = torch.cat([torch.zeros_like(w), cross(vp, w)], -1)
        else:
            Vpar = V[par] if par >= 0 else torch.zeros(B, 6, dtype=F64)
            Sdot_qd = mcross(Vpar, S[j][:, :, 0]) * qdj
        Apar = A[par] if par >= 0 else torch.zeros(B, 6, dtype=F64)
        A.append(Apar + Sdot_qd)                 # Jdot_j qd
    bl = m.bodies
    Rb = torch.stack([R[j] for j in bl], 1)       # [B,nb,3,3]
    pb = torch.stack([p[j] for j in bl], 1)
    mass = m.mass[bl]                             # [nb]
    c = pb + (Rb @ m.com[bl][None, :, :, None])[..., 0]
    Ic = Rb @ m.inertia[bl][None] @ Rb.transpose(-1, -2)
    C = skew(c)
    eye = torch.eye(3, dtype=F64).expand(C.shape)
    mm = mass[None, :, None, None]
    I6 = torch.cat([torch.cat([Ic + mm * (C @ C.transpose(-1, -2)), mm * C], -1),
                    torch.cat([mm * C.transpose(-1, -2), mm * eye], -1)], -2)   # [B,nb,6,6]
    Jbb = torch.stack([Jb[j] for j in bl], 1)     # [B,nb,6,nv]
    Vb = torch.stack([V[j] for j in bl], 1)
    Ab = torch.stack([A[j] for j in bl], 1)
    a_g = torch.tensor([0.0, 0.0, 0.0, 0.0, 0.0, -m.g], dtype=F64)
    M = (Jbb.transpose(-1, -2) @ I6 @ Jbb).sum(1) + torch.diag(m.armature)
    hb = (I6 @ Vb[..., None])[..., 0]
    fb = (I6 @ (Ab - a_g)[..., None])[..., 0] + fcross(Vb, hb)
    bias = (Jbb.transpose(-1, -2) @ fb[..., None])[..., 0].sum(1)
    out = dict(R=R, p=p, S=S, Jb=Jb, V=V, A=A, M=M, bias=bias, I6=I6, bodies=bl)
    # contacts
    if len(m.cbody) > 0:
        cb = m.cbody
        Rc = torch.stack([R[j] for j in cb], 1)
        pc = torch.stack([p[j] for j in cb], 1)
        Jc = torch.stack([Jb[j] for j in cb], 1)                       # [B,nc,6,nv]
        xc = pc + (Rc @ m.cpos[None, :, :, None])[..., 0]             # sphere centres
        zhat = torch.tensor([0.0, 0.0, 1.0], dtype=F64)
        xp = xc - m.crad[None, :, None] * zhat                        # contact points
        Jpt = Jc[:, :, 3:, :] - skew(xp) @ Jc[:, :, :3, :]             # point Jacobians
        vpt = (Jpt @ qd[:, None, :, None])[..., 0]
        d = xc[..., 2] - m.crad[None, :]
        ddot = vpt[..., 2]
        pen = torch.where(d < 0.0, d, torch.zeros_like(d))
        fn = (-m.kn + m.kd * ddot) * pen
        vt = torch.cat([vpt[..., :2], torch.zeros_like(vpt[..., 2:])], -1)
        vt2 = (vt * vt).sum(-1)
        afn = torch.abs(fn)
        viscous = (m.kt * m.kt * vt2) <= (m.mu * afn) ** 2
        vn = torch.sqrt(torch.where(viscous, torch.ones_like(vt2), vt2))
        ft = torch.where(viscous[..., None], -m.kt * vt, -(m.mu * afn / vn)[..., None] * vt)
        ft = torch.where((d < 0.0)[..., None], ft, torch.zeros_like(ft))
        f = ft + fn[..., None] * zhat
        tau_c = (Jpt.transpose(-1, -2) @ f[..., None])[..., 0].sum(1)
        out.update(contact_x=xp, contact_d=d, contact_f=f, contact_v=vpt, tau_contact=tau_c)
    else:
        out["tau_contact"] = torch.zeros(B, m.nv, dtype=F64)
    return out


def muscle_terms(m, T, qd, act):
    """Generalized forces of the muscle-tendon units at activation ``act`` [B, n_mtu],
    with the path lengths, rates and tensions (point Jacobians as for the contacts)."""
    B = qd.shape[0]
    Rall = torch.stack(T["R"], 1)                                     # [B,J,3,3]
    pall = torch.stack(T["p"], 1)
    Jall = torch.stack(T["Jb"], 1)                                    # [B,J,6,nv]
    bi = m.mtu_body                                                   # [n,P]
    x = pall[:, bi] + (Rall[:, bi] @ m.mtu_pos[None, :, :, :, None])[..., 0]      # [B,n,P,3]
    Jp = Jall[:, bi]                                                  # [B,n,P,6,nv]
    Jpt = Jp[..., 3:, :] - skew(x) @ Jp[..., :3, :]                   # point Jacobians
    v = (Jpt @ qd[:, None, None, :, None])[..., 0]                    # [B,n,P,3]
    seg_ok = (m.mtu_valid[:, 1:] & m.mtu_valid[:, :-1]).to(F64)       # [n,P-1]
    # segments past a path's last point get a unit dummy vector (masked out below), so
    # that no square root is taken at zero length
    dummy = torch.tensor([1.0, 0.0, 0.0], dtype=F64)
    d = (x[:, :, 1:] - x[:, :, :-1]) * seg_ok[..., None] + (1.0 - seg_ok)[..., None] * dummy
    ell = torch.sqrt((d * d).sum(-1))
    u = d / ell[..., None] * seg_ok[..., None]                        # unit segment vectors
    L = (ell * seg_ok).sum(-1)                                         # [B,n]
    Ldot = (u * (v[:, :, 1:] - v[:, :, :-1])).sum(-1).sum(-1)
    lm = L - m.mtu_lslack
    fl = torch.exp(-(((lm / m.mtu_lopt) - 1.0) / m.fl_width) ** 2)
    fv = 1.0 + Ldot / (m.vmax * m.mtu_lopt)
    F = torch.clamp(m.mtu_fmax * act * fl * fv, min=0.0)
    # point forces F (u_k - u_{k-1}), u_{-1} = u_last = 0 (masked)
    z = torch.zeros_like(u[:, :, :1])
    uf = torch.cat([u, z], 2)
    ub = torch.cat([z, u], 2)
    fpt = F[..., None, None] * (uf - ub)                               # [B,n,P,3]
    tau = (Jpt.transpose(-1, -2) @ fpt[..., None])[..., 0].sum((1, 2))
    return dict(tau=tau, L=L, Ldot=Ldot, F=F, x=x, fpt=fpt)


def activation_step(m, act, u, dt):
    """First-order activation lag, explicit over one substep."""
    return act + dt * (u - act) / m.tau_act


def joint_torques(m, q, a):
    """Actuation gear * a plus the joint-limit penalty, in velocity coordinates."""
    B = q.shape[0]
    cols = [torch.zeros(B, dtype=F64) for _ in range(m.nv)]
    for i, j in enumerate(m.act_joint):                 # motors are the first actions
        cols[m.vadr[j]] = cols[m.vadr[j]] + m.gear[i] * a[:, i]
    for j in range(m.J):
        if m.limited[j] and m.jtype[j] != FREE:
            qj = q[:, m.qadr[j]]
            lo, hi = m.lower[j], m.upper[j]
            t = torch.where(qj < lo, m.klim * (lo - qj),
                            torch.where(qj > hi, m.klim * (hi - qj), torch.zeros_like(qj)))
            cols[m.vadr[j]] = cols[m.vadr[j]] + t
    return torch.stack(cols, 1)


def integrate(m, q, qd_new, dt):
    """Semi-implicit Euler position update with the already-updated velocities."""
    parts = []
    for j in range(m.J):
        a, v = m.qadr[j], m.vadr[j]
        if m.jtype[j] == FREE:
            parts.append(q[:, a:a + 3] + dt * qd_new[:, v:v + 3])
            parts.append(quat_exp_update(q[:, a + 3:a + 7], qd_new[:, v + 3:v + 6], dt))
        else:
            parts.append(q[:, a:a + 1] + dt * qd_new[:, v:v + 1])
    return torch.cat(parts, 1)


def substep(m, q, qd, a, dt, act=None, stats=None):
    """One semi-implicit Euler substep of M qdd = J^T f + c + tau (Sec. 3.1).  Muscle
    models also take the activations ``act`` and return the updated ones.  ``stats``, a
    list, receives per env the number of contacts that penetrate with a pulling normal
    force (the literal damping term exceeding the stiffness term)."""
    T = dynamics_terms(m, q, qd)
    if stats is not None and "contact_d" in T:
        stats.append(((T["contact_d"] < 0.0) & (T["contact_f"][..., 2] < 0.0)).sum(1))
    tau = joint_torques(m, q, a) + T["tau_contact"] - T["bias"]
    if m.n_mtu:
        tau = tau + muscle_terms(m, T, qd, act)["tau"]
    L = torch.linalg.cholesky(T["M"])
    qdd = torch.cholesky_solve(tau[..., None], L)[..., 0]
    qd_new = qd + dt * qdd
    if m.n_mtu:
        act_new = activation_step(m, act, a[:, m.n_motor:], dt)
        return integrate(m, q, qd_new, dt), qd_new, act_new
    return integrate(m, q, qd_new, dt), qd_new


def kinetic_energy(m, q, qd):
    T = dynamics_terms(m, q, qd)
    return 0.5 * (qd[:, None, :] @ T["M"] @ qd[:, :, None])[:, 0, 0], T


def potential_energy(m, q):
    R, p = forward_kinematics(m, q)
    e = torch.zeros(q.shape[0], dtype=F64)
    for j in m.bodies:
        cz = (p[j] + R[j] @ m.com[j])[:, 2]
        e = e + m.mass[j] * m.g * cz
    return e
