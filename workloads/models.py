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
                   root_height=h0, has_last_action=1)


def humanoid(seed=0):
    """13 capsule bodies on a free root plus 21 hinges (abdomen 3, hip 3, knee 1,
    ankle 2 per leg, shoulder 2, elbow 1 per arm; 9 massless intermediate frames),
    body masses U(1, 8) kg from ``seed``, gear 25..100, 10 contact spheres (4 foot
    capsule ends, 2 knees, 2 hands, pelvis, head)."""
    rng = np.random.default_rng(seed)
    masses = rng.uniform(1.0, 8.0, 13)
    mi = iter(masses)
    b = _Builder("humanoid", "humanoid")
    arm = 0.02

    def cap(p0, p1, r):
        m = next(mi)
        c, I = capsule_inertia(m, p0, p1, r)
        return dict(mass=m, com=c, inertia=I)

    root = b.joint(-1, FREE, name="root", **cap((0, 0, -0.05), (0, 0, 0.15), 0.09))
    b.contact(root, (0, 0, 0.19), 0.09)                                   # head
    az = b.joint(root, HINGE, offset=(-0.01, 0, -0.26), axis=(0, 0, 1), limit=(-0.8, 0.8),
                 gear=75, armature=arm, name="abdomen_z")
    ay = b.joint(az, HINGE, axis=(0, 1, 0), limit=(-1.3, 0.5), gear=75, armature=arm,
                 name="abdomen_y", **cap((0, -0.06, 0), (0, 0.06, 0), 0.06))
    pel = b.joint(ay, HINGE, offset=(0, 0, -0.165), axis=(1, 0, 0), limit=(-0.6, 0.6), gear=75,
                  armature=arm, name="abdomen_x", **cap((-0.02, -0.07, 0), (-0.02, 0.07, 0), 0.09))
    b.contact(pel, (-0.02, 0, 0), 0.09)                                   # pelvis
    for s in (1.0, -1.0):                                                 # right, left
        hx = b.joint(pel, HINGE, offset=(0, -0.1 * s, -0.04), axis=(s, 0, 0), limit=(-0.6, 0.4),
                     gear=100, armature=arm, name="hip_x")
        hz = b.joint(hx, HINGE, axis=(0, 0, s), limit=(-1.0, 0.6), gear=100, armature=arm,
                     name="hip_z")
        hy = b.joint(hz, HINGE, axis=(0, 1, 0), limit=(-1.9, 0.35), gear=100, armature=arm,
                     name="hip_y", **cap((0, 0, 0), (0, 0.01 * s, -0.34), 0.06))
        kn = b.joint(hy, HINGE, offset=(0, 0.01 * s, -0.403), axis=(0, -1, 0), limit=(-0.35, 2.8),
                     gear=100, armature=arm, name="knee", **cap((0, 0, 0), (0, 0, -0.3), 0.049))
        b.contact(kn, (0, 0, 0), 0.06)                                    # knee
        ky = b.joint(kn, HINGE, offset=(0, 0, -0.39), axis=(0, 1, 0), limit=(-0.8, 0.8),
                     gear=50, armature=arm, name="ankle_y")
        ft = b.joint(ky, HINGE, axis=(s, 0, 0), limit=(-0.6, 0.6), gear=50, armature=arm,
                     name="ankle_x", **cap((-0.04, 0, -0.05), (0.12, 0, -0.05), 0.04))
        b.contact(ft, (-0.04, 0, -0.05), 0.04)                            # heel
        b.contact(ft, (0.12, 0, -0.05), 0.04)                             # toe
    for s in (1.0, -1.0):
        s1 = b.joint(root, HINGE, offset=(0, -0.17 * s, 0.06), axis=(2, s, 1), limit=(-1.5, 1.0),
                     gear=25, armature=arm, name="shoulder1")
        s2 = b.joint(s1, HINGE, axis=(0, -s, 1), limit=(-1.5, 1.0), gear=25, armature=arm,
                     name="shoulder2", **cap((0, 0, 0), (0.16, -0.16 * s, -0.16), 0.04))
        el = b.joint(s2, HINGE, offset=(0.18, -0.18 * s, -0.18), axis=(0, -s, 1),
                     limit=(-1.6, 0.8), gear=25, armature=arm, name="elbow",
                     **cap((0.01, 0.01 * s, 0.01), (0.17, 0.17 * s, 0.17), 0.031))
        b.contact(el, (0.18, 0.18 * s, 0.18), 0.04)                      # hand
    # root height at which the foot spheres touch the ground with every hinge at 0
    h0 = 0.26 + 0.165 + 0.04 + 0.403 + 0.39 + 0.05 + 0.04
    return b.build(substeps=48, kn=4.0e4, kd=1.0e4, kt=1.0e3, mu=0.75, klim=1.0e4,
                   root_height=h0, has_last_action=1)


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


def model_by_name(name):
    return {"cartpole": cartpole, "ant": ant, "humanoid": humanoid}[name]()
