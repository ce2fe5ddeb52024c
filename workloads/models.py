"""Articulated-body model descriptions (data only).

A model is a tree of joint frames.  Frame j hangs from frame parent[j]
(-1 = the world) at a fixed offset expressed in the parent frame, with no fixed
rotation, and then moves through its own joint:

* FREE  - 7 position coordinates (x, y, z, qw, qx, qy, qz), 6 velocity
          coordinates (world linear velocity of the frame origin, world angular
          velocity).  Only allowed for a root frame.
* HINGE - one angle about ``axis`` (a unit vector in the frame).
* SLIDE - one displacement along ``axis``.

Each frame may carry a rigid body (mass, centre of mass and rotational inertia
about the centre of mass, both in the frame) and contact spheres.  A frame
with zero mass is a massless intermediate frame of a multi-axis joint.

The world is z-up with the ground plane at z = 0.  The numbers in this module
are the synthetic morphologies that stand in for the paper's task models,
which are not available (CartPole, Ant and Humanoid of the benchmark tasks).
"""
import numpy as np

FREE, HINGE, SLIDE = 0, 1, 2

DT_FRAME = 1.0 / 60.0


class _Builder:
    def __init__(self, name, task):
        self.name, self.task = name, task
        self.rows = []
        self.contacts = []

    def joint(self, parent, jtype, offset=(0, 0, 0), axis=(0, 0, 1), mass=0.0,
              com=(0, 0, 0), inertia=None, limit=None, gear=0.0, armature=0.0,
              q_mean=0.0, name=""):
        ax = np.asarray(axis, float)
        ax = ax / np.linalg.norm(ax)
        self.rows.append(dict(parent=parent, jtype=jtype, offset=np.asarray(offset, float),
                              axis=ax, mass=float(mass), com=np.asarray(com, float),
                              inertia=np.zeros((3, 3)) if inertia is None else np.asarray(inertia, float),
                              limit=limit, gear=float(gear), armature=float(armature),
                              q_mean=float(q_mean), name=name))
        return len(self.rows) - 1

    def contact(self, body, pos, radius):
        self.contacts.append((body, np.asarray(pos, float), float(radius)))

    def build(self, **params):
        J = len(self.rows)
        nq = nv = 0
        qadr, vadr = [], []
        for r in self.rows:
            qadr.append(nq)
            vadr.append(nv)
            if r["jtype"] == FREE:
                nq += 7
                nv += 6
            else:
                nq += 1
                nv += 1
        act = [j for j, r in enumerate(self.rows) if r["gear"] != 0.0]
        armature = np.zeros(nv)
        for j, r in enumerate(self.rows):
            if r["jtype"] != FREE:
                armature[vadr[j]] = r["armature"]
        m = dict(
            name=self.name, task=self.task,
            n_joints=J, nq=nq, nv=nv, na=len(act),
            parent=np.array([r["parent"] for r in self.rows], np.int32),
            jtype=np.array([r["jtype"] for r in self.rows], np.int32),
            qadr=np.array(qadr, np.int32), vadr=np.array(vadr, np.int32),
            offset=np.stack([r["offset"] for r in self.rows]),
            axis=np.stack([r["axis"] for r in self.rows]),
            mass=np.array([r["mass"] for r in self.rows]),
            com=np.stack([r["com"] for r in self.rows]),
            inertia=np.stack([r["inertia"] for r in self.rows]),
            limited=np.array([r["limit"] is not None for r in self.rows], np.int32),
            lower=np.array([r["limit"][0] if r["limit"] is not None else 0.0 for r in self.rows]),
            upper=np.array([r["limit"][1] if r["limit"] is not None else 0.0 for r in self.rows]),
            q_mean=np.array([r["q_mean"] for r in self.rows]),
            act_joint=np.array(act, np.int32),
            gear=np.array([self.rows[j]["gear"] for j in act]),
            armature=armature,
            contact_body=np.array([c[0] for c in self.contacts], np.int32),
            contact_pos=np.stack([c[1] for c in self.contacts]) if self.contacts else np.zeros((0, 3)),
            contact_radius=np.array([c[2] for c in self.contacts]),
            joint_names=[r["name"] for r in self.rows],
        )
        for j, r in enumerate(self.rows):
            assert r["parent"] < j, "frames must be listed parents first"
            assert r["jtype"] != FREE or r["parent"] == -1, "FREE joints must be roots"
        m.update(n_motor=len(act), n_mtu=0)
        base = dict(gravity=9.81, kn=0.0, kd=0.0, kt=0.0, mu=0.0, klim=0.0,
                    dt=DT_FRAME, substeps=1, root_height=0.0, has_last_action=0)
        base.update(params)
        m.update(base)
        return m


# ---------------------------------------------------------------- inertias

def capsule_inertia(mass, p0, p1, radius):
    """Solid capsule (cylinder p0-p1 plus two hemispherical caps) of uniform density.

    Returns (com, inertia about the com) in the frame of p0/p1.
    """
    p0, p1 = np.asarray(p0, float), np.asarray(p1, float)
    seg = p1 - p0
    L = float(np.linalg.norm(seg))
    r = float(radius)
    v_cyl = np.pi * r * r * L
    v_sph = 4.0 / 3.0 * np.pi * r ** 3
    m_cyl = mass * v_cyl / (v_cyl + v_sph)
    m_sph = mass - m_cyl
    i_ax = m_cyl * r * r / 2.0 + m_sph * 2.0 / 5.0 * r * r
    i_perp = (m_cyl * (r * r / 4.0 + L * L / 12.0)
              + m_sph * (83.0 / 320.0 * r * r + (L / 2.0 + 3.0 * r / 8.0) ** 2))
    u = seg / L if L > 0 else np.array([0.0, 0.0, 1.0])
    inertia = i_perp * (np.eye(3) - np.outer(u, u)) + i_ax * np.outer(u, u)
    return (p0 + p1) / 2.0, inertia


def sphere_inertia(mass, radius):
    return 2.0 / 5.0 * mass * radius * radius * np.eye(3)


# ---------------------------------------------------------------- task models

def cartpole():
    """Cart (1 kg) on a slide along x, pole (uniform 1 m rod, 0.1 kg) on a hinge about y.

    Pole angle 0 is upright; the cart force is gear 1 N per unit action.
    """
    b = _Builder("cartpole", "cartpole")
    cart = b.joint(-1, SLIDE, axis=(1, 0, 0), mass=1.0,
                   inertia=np.diag([0.01, 0.01, 0.01]), gear=1.0, name="slider")
    mp, L = 0.1, 1.0
    b.joint(cart, HINGE, axis=(0, 1, 0), mass=mp, com=(0, 0, L / 2),
            inertia=np.diag([mp * L * L / 12.0, mp * L * L / 12.0, 0.0]), name="hinge")
    return b.build(substeps=4)


def ant():
    """Quadruped: 0.5 kg sphere torso (r 0.25) on a free base, four legs of two
    capsules (0.2 m / 0.4 m, r 0.08, 1.0 kg / 1.5 kg), hip about z (+-30 deg),
    knee about the horizontal axis normal to the leg (30..70 deg, positive bends
    down), gear 50, contact spheres at the distal end of each leg capsule."""
    b = _Builder("ant", "ant")
    r_leg = 0.08
    torso = b.joint(-1, FREE, mass=0.5, inertia=sphere_inertia(0.5, 0.25), name="root")
    d30, d50, d70 = np.deg2rad(30.0), np.deg2rad(50.0), np.deg2rad(70.0)
    for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        d = np.array([sx, sy, 0.0]) / np.sqrt(2.0)
        com_u, in_u = capsule_inertia(1.0, (0, 0, 0), 0.2 * d, r_leg)
        hip = b.joint(torso, HINGE, offset=0.25 * d, axis=(0, 0, 1), mass=1.0, com=com_u,
                      inertia=in_u, limit=(-d30, d30), gear=50.0, armature=0.1, name="hip")
        b.contact(hip, 0.2 * d, r_leg)
        knee_axis = np.cross([0.0, 0.0, 1.0], d)
        com_l, in_l = capsule_inertia(1.5, (0, 0, 0), 0.4 * d, r_leg)
        knee = b.joint(hip, HINGE, offset=0.2 * d, axis=knee_axis, mass=1.5, com=com_l,
                       inertia=in_l, limit=(d30, d70), gear=50.0, armature=0.1,
                       q_mean=d50, name="knee")
        b.contact(knee, 0.4 * d, r_leg)
    # torso height at which the lowest contact sphere touches the ground with the
    # knees at their mean angle (lower leg tilted down by d50)
    h0 = 0.4 * np.sin(d50) + r_leg
    return b.build(substeps=16, kn=4.0e4, kd=1.0e4, kt=1.0e3, mu=0.75, klim=1.0e4,
                   root_height=h0, has_last_action=1, et_height=0.27)


def _humanoid_frames(b, rng, motors=True):
    """The humanoid skeleton of ``humanoid`` on builder ``b``.  Returns the body frames by
    name and each body's capsule (p0, p1, r) in its frame.  Joint motors are added only
    when ``motors``."""
    masses = rng.uniform(1.0, 8.0, 13)
    mi = iter(masses)
    arm = 0.02
    caps = {}
    names = {}

    def g(x):
        return x if motors else 0.0

    def cap(p0, p1, r):
        m = next(mi)
        c, I = capsule_inertia(m, p0, p1, r)
        return dict(mass=m, com=c, inertia=I), (np.asarray(p0, float), np.asarray(p1, float), float(r))

    kw, cp = cap((0, 0, -0.05), (0, 0, 0.15), 0.09)
    root = b.joint(-1, FREE, name="root", **kw)
    caps[root] = cp
    names["torso"] = root
    b.contact(root, (0, 0, 0.19), 0.09)                                   # head
    az = b.joint(root, HINGE, offset=(-0.01, 0, -0.26), axis=(0, 0, 1), limit=(-0.8, 0.8),
                 gear=g(75), armature=arm, name="abdomen_z")
    kw, cp = cap((0, -0.06, 0), (0, 0.06, 0), 0.06)
    ay = b.joint(az, HINGE, axis=(0, 1, 0), limit=(-1.3, 0.5), gear=g(75), armature=arm,
                 name="abdomen_y", **kw)
    caps[ay] = cp
    names["lwaist"] = ay
    kw, cp = cap((-0.02, -0.07, 0), (-0.02, 0.07, 0), 0.09)
    pel = b.joint(ay, HINGE, offset=(0, 0, -0.165), axis=(1, 0, 0), limit=(-0.6, 0.6), gear=g(75),
                  armature=arm, name="abdomen_x", **kw)
    caps[pel] = cp
    names["pelvis"] = pel
    b.contact(pel, (-0.02, 0, 0), 0.09)                                   # pelvis
    for s, side in ((1.0, "r"), (-1.0, "l")):
        hx = b.joint(pel, HINGE, offset=(0, -0.1 * s, -0.04), axis=(s, 0, 0), limit=(-0.6, 0.4),
                     gear=g(100), armature=arm, name="hip_x")
        hz = b.joint(hx, HINGE, axis=(0, 0, s), limit=(-1.0, 0.6), gear=g(100), armature=arm,
                     name="hip_z")
        kw, cp = cap((0, 0, 0), (0, 0.01 * s, -0.34), 0.06)
        hy = b.joint(hz, HINGE, axis=(0, 1, 0), limit=(-1.9, 0.35), gear=g(100), armature=arm,
                     name="hip_y", **kw)
        caps[hy] = cp
        names["thigh_" + side] = hy
        kw, cp = cap((0, 0, 0), (0, 0, -0.3), 0.049)
        kn = b.joint(hy, HINGE, offset=(0, 0.01 * s, -0.403), axis=(0, -1, 0), limit=(-0.35, 2.8),
                     gear=g(100), armature=arm, name="knee", **kw)
        caps[kn] = cp
        names["shin_" + side] = kn
        b.contact(kn, (0, 0, 0), 0.06)                                    # knee
        ky = b.joint(kn, HINGE, offset=(0, 0, -0.39), axis=(0, 1, 0), limit=(-0.8, 0.8),
                     gear=g(50), armature=arm, name="ankle_y")
        kw, cp = cap((-0.04, 0, -0.05), (0.12, 0, -0.05), 0.04)
        ft = b.joint(ky, HINGE, axis=(s, 0, 0), limit=(-0.6, 0.6), gear=g(50), armature=arm,
                     name="ankle_x", **kw)
        caps[ft] = cp
        names["foot_" + side] = ft
        b.contact(ft, (-0.04, 0, -0.05), 0.04)                            # heel
        b.contact(ft, (0.12, 0, -0.05), 0.04)                             # toe
    for s, side in ((1.0, "r"), (-1.0, "l")):
        s1 = b.joint(root, HINGE, offset=(0, -0.17 * s, 0.06), axis=(2, s, 1), limit=(-1.5, 1.0),
                     gear=g(25), armature=arm, name="shoulder1")
        kw, cp = cap((0, 0, 0), (0.16, -0.16 * s, -0.16), 0.04)
        s2 = b.joint(s1, HINGE, axis=(0, -s, 1), limit=(-1.5, 1.0), gear=g(25), armature=arm,
                     name="shoulder2", **kw)
        caps[s2] = cp
        names["uarm_" + side] = s2
        kw, cp = cap((0.01, 0.01 * s, 0.01), (0.17, 0.17 * s, 0.17), 0.031)
        el = b.joint(s2, HINGE, offset=(0.18, -0.18 * s, -0.18), axis=(0, -s, 1),
                     limit=(-1.6, 0.8), gear=g(25), armature=arm, name="elbow", **kw)
        caps[el] = cp
        names["larm_" + side] = el
        b.contact(el, (0.18, 0.18 * s, 0.18), 0.04)                      # hand
    return names, caps


# root height at which the foot spheres touch the ground with every hinge at 0
_HUMANOID_H0 = 0.26 + 0.165 + 0.04 + 0.403 + 0.39 + 0.05 + 0.04


def humanoid(seed=0):
    """13 capsule bodies on a free root plus 21 hinges (abdomen 3, hip 3, knee 1,
    ankle 2 per leg, shoulder 2, elbow 1 per arm; 9 massless intermediate frames),
    body masses U(1, 8) kg from ``seed``, gear 25..100, 10 contact spheres (4 foot
    capsule ends, 2 knees, 2 hands, pelvis, head)."""
    rng = np.random.default_rng(seed)
    b = _Builder("humanoid", "humanoid")
    _humanoid_frames(b, rng, motors=True)
    return b.build(substeps=48, kn=4.0e4, kd=1.0e4, kt=1.0e3, mu=0.75, klim=1.0e4,
                   root_height=_HUMANOID_H0, has_last_action=1, et_height=0.74)


# Muscle groups of the muscle-driven humanoid: (origin body, insertion body, count,
# F_max range in N).  Lower-body heavy, with one- and two-joint muscles; "*" = each side.
MTU_GROUPS = [
    ("torso", "lwaist", 8, (200.0, 800.0)),
    ("lwaist", "pelvis", 8, (200.0, 800.0)),
    ("torso", "pelvis", 12, (200.0, 800.0)),
    ("pelvis", "thigh_*", 24, (300.0, 1200.0)),
    ("thigh_*", "shin_*", 10, (300.0, 1200.0)),
    ("pelvis", "shin_*", 8, (300.0, 1200.0)),
    ("shin_*", "foot_*", 10, (200.0, 900.0)),
    ("thigh_*", "foot_*", 4, (200.0, 900.0)),
    ("torso", "uarm_*", 4, (50.0, 300.0)),
    ("uarm_*", "larm_*", 2, (50.0, 300.0)),
]
MTU_MAX_POINTS = 6


def _rest_origins(md):
    """World origin of every frame in the rest pose (root at the origin, hinges at 0)."""
    o = np.zeros((md["n_joints"], 3))
    for j in range(md["n_joints"]):
        par = md["parent"][j]
        if par >= 0:
            o[j] = o[par] + md["offset"][j]
    return o


def mtu_humanoid(seed=0):
    """The humanoid skeleton (same bodies, masses and contacts as ``humanoid``) with no
    joint motors, driven by 152 Hill-type muscle-tendon units.  Each unit is a polyline
    from an origin on one body through 2..4 via points to an insertion on a body further
    down the tree; every point is fixed in a body frame.  Per unit: F_max, optimal fibre
    length l_opt and tendon slack length l_slack, chosen so that the rest pose has
    l_m / l_opt in [0.9, 1.1].  Actions are the 152 excitations; activations follow a
    first-order lag (tau 10 ms) and are part of the state."""
    b = _Builder("mtu_humanoid", "mtu")
    names, caps = _humanoid_frames(b, np.random.default_rng(seed), motors=False)
    md = b.build(substeps=48, kn=4.0e4, kd=1.0e4, kt=1.0e3, mu=0.75, klim=1.0e4,
                 root_height=_HUMANOID_H0, has_last_action=0, et_height=0.74)
    rng = np.random.default_rng([seed, 1])
    origin = _rest_origins(md)
    parent = md["parent"]

    def chain(a, bb):
        path = [bb]
        while path[-1] != a:
            path.append(int(parent[path[-1]]))
        return [j for j in reversed(path) if j in caps]

    def surface_point(j):
        p0, p1, r = caps[j]
        ax = p1 - p0
        t = rng.uniform(0.2, 0.8)
        u = ax / max(np.linalg.norm(ax), 1e-9)
        d = rng.normal(size=3)
        d -= u * (d @ u)
        d /= np.linalg.norm(d)
        return p0 + t * ax + r * rng.uniform(0.9, 1.3) * d

    bodies, pos, npt, fmax, lopt, lslack = [], [], [], [], [], []
    for a_name, b_name, count, (flo, fhi) in MTU_GROUPS:
        sides = ("r", "l") if "*" in a_name + b_name else ("",)
        for side in sides:
            A = names[a_name.replace("*", side)]
            B = names[b_name.replace("*", side)]
            ch = chain(A, B)
            for _ in range(count):
                pa, pb = surface_point(A), surface_point(B)
                wa, wb = origin[A] + pa, origin[B] + pb
                bulge = rng.normal(size=3)
                dab = wb - wa
                bulge -= dab * (bulge @ dab) / (dab @ dab)
                bulge *= 0.03 / np.linalg.norm(bulge)
                K = int(rng.integers(2, 5))
                pts = [(A, pa)]
                for k in range(1, K + 1):
                    f = k / (K + 1.0)
                    w = wa + f * dab + bulge * np.sin(np.pi * f)
                    # attach to the chain body whose capsule is nearest in the rest pose
                    best, bd = ch[0], np.inf
                    for j in ch:
                        p0, p1, _ = caps[j]
                        s0, s1 = origin[j] + p0, origin[j] + p1
                        sg = s1 - s0
                        tt = np.clip((w - s0) @ sg / max(sg @ sg, 1e-12), 0.0, 1.0)
                        dist = np.linalg.norm(w - (s0 + tt * sg))
                        if dist < bd:
                            best, bd = j, dist
                    pts.append((best, w - origin[best]))
                pts.append((B, pb))
                world = np.array([origin[j] + r for j, r in pts])
                L0 = float(np.linalg.norm(np.diff(world, axis=0), axis=1).sum())
                ls = rng.uniform(0.2, 0.5) * L0
                lo = (L0 - ls) / rng.uniform(0.9, 1.1)
                bodies.append([j for j, _ in pts] + [0] * (MTU_MAX_POINTS - len(pts)))
                pos.append([r for _, r in pts] + [np.zeros(3)] * (MTU_MAX_POINTS - len(pts)))
                npt.append(len(pts))
                fmax.append(rng.uniform(flo, fhi))
                lopt.append(lo)
                lslack.append(ls)
    n = len(npt)
    md.update(n_mtu=n, n_motor=0, na=n,
              mtu_npt=np.array(npt, np.int32), mtu_body=np.array(bodies, np.int32),
              mtu_pos=np.array(pos, float), mtu_fmax=np.array(fmax), mtu_lopt=np.array(lopt),
              mtu_lslack=np.array(lslack), tau_act=0.01, fl_width=0.45, vmax=10.0)
    return md


# ---------------------------------------------------------------- small test models

def pendulum(mass=0.1, length=1.0):
    """Uniform rod on a world hinge about y, angle 0 hanging straight down."""
    b = _Builder("pendulum", "none")
    b.joint(-1, HINGE, axis=(0, 1, 0), mass=mass, com=(0, 0, -length / 2),
            inertia=np.diag([mass * length ** 2 / 12, mass * length ** 2 / 12, 0.0]), gear=1.0)
    return b.build()


def free_body(mass=2.0, inertia=(0.1, 0.2, 0.3), radius=0.1, gravity=9.81, contact=False, **kw):
    """A single free rigid body, optionally with one contact sphere at its origin."""
    b = _Builder("free_body", "none")
    r = b.joint(-1, FREE, mass=mass, inertia=np.diag(inertia))
    if contact:
        b.contact(r, (0, 0, 0), radius)
    return b.build(gravity=gravity, **kw)


def sliding_block(mass=1.0, radius=0.05, **kw):
    """A free body with four contact spheres at its base corners."""
    b = _Builder("sliding_block", "none")
    r = b.joint(-1, FREE, mass=mass, inertia=np.diag([0.01, 0.01, 0.01]))
    for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        b.contact(r, (0.1 * sx, 0.1 * sy, 0.0), radius)
    return b.build(**kw)


def chain(n=3, free_root=True, seed=7, gravity=9.81, **kw):
    """A random serial/branched chain of capsules, for identity checks."""
    rng = np.random.default_rng(seed)
    b = _Builder("chain", "none")
    if free_root:
        root = b.joint(-1, FREE, mass=1.0, inertia=np.diag([0.05, 0.06, 0.07]))
    else:
        root = b.joint(-1, HINGE, axis=rng.normal(size=3), mass=1.0,
                       com=rng.normal(size=3) * 0.1, inertia=np.diag([0.05, 0.06, 0.07]),
                       gear=1.0)
    prev = root
    for i in range(n):
        par = prev if (i % 2 == 0 or i < 2) else root
        off = rng.normal(size=3) * 0.2
        tip = rng.normal(size=3) * 0.2
        m = rng.uniform(0.5, 2.0)
        c, I = capsule_inertia(m, (0, 0, 0), tip, 0.05)
        jt = SLIDE if (i == 1) else HINGE
        prev = b.joint(par, jt, offset=off, axis=rng.normal(size=3), mass=m,
                       com=c, inertia=I, gear=1.0)
    return b.build(gravity=gravity, **kw)


def muscle_arm(d=0.3, b=0.8, c=None, fmax=50.0, lopt=0.6, lslack=0.2):
    """Cart on a slide along x (1 kg) with a pole hinged about y (uniform 1 m rod, 0.5 kg,
    angle 0 upright), one muscle from the cart at (d, 0, 0) to the pole at height b
    (through a via point on the pole at height c if given).  No gravity, so the muscle is
    the only load.  Path length: L(theta) = sqrt(b^2 + d^2 - 2 b d sin theta), or with the
    via point sqrt(c^2 + d^2 - 2 c d sin theta) + (b - c)."""
    bld = _Builder("muscle_arm", "none")
    cart = bld.joint(-1, SLIDE, axis=(1, 0, 0), mass=1.0, inertia=np.diag([0.01, 0.01, 0.01]),
                     name="slider")
    mp, Lp = 0.5, 1.0
    pole = bld.joint(cart, HINGE, axis=(0, 1, 0), mass=mp, com=(0, 0, Lp / 2),
                     inertia=np.diag([mp * Lp * Lp / 12.0, mp * Lp * Lp / 12.0, 0.0]), name="hinge")
    md = bld.build(substeps=4, gravity=0.0)
    pts = [(cart, (d, 0.0, 0.0))]
    if c is not None:
        pts.append((pole, (0.0, 0.0, c)))
    pts.append((pole, (0.0, 0.0, b)))
    n = len(pts)
    body = [j for j, _ in pts] + [0] * (MTU_MAX_POINTS - n)
    pos = [np.asarray(r, float) for _, r in pts] + [np.zeros(3)] * (MTU_MAX_POINTS - n)
    md.update(n_mtu=1, n_motor=0, na=1, mtu_npt=np.array([n], np.int32),
              mtu_body=np.array([body], np.int32), mtu_pos=np.array([pos], float),
              mtu_fmax=np.array([fmax]), mtu_lopt=np.array([lopt]), mtu_lslack=np.array([lslack]),
              tau_act=0.01, fl_width=0.45, vmax=10.0)
    return md


def model_by_name(name):
    return {"cartpole": cartpole, "ant": ant, "humanoid": humanoid, "mtu_humanoid": mtu_humanoid}[name]()


def with_termination(md):
    """A copy of a floating-base model with early termination at its task's root height
    (App. A.3: Ant 0.27 m, Humanoid torso 0.74 m; the muscle humanoid shares the humanoid's
    skeleton and root, so it takes the same height)."""
    d = dict(md)
    d["term_height"] = float(md["et_height"])
    return d
