"""Seeded initial states, MLP weights and named workload configurations (data only).

State layout (one row per env, env-major):  s = [q (nq) | qd (nv) | a_prev (na, only
for tasks whose observation holds the last action) | muscle activations (n_mtu, muscle
models only)].
"""
import numpy as np

from .models import FREE, model_by_name

# network sizes: actor / critic hidden layers (paper's network table; the Ant actor
# follows the benchmark configuration 37-128-64-8)
NETS = {
    "cartpole": ([64, 64], [64, 64]),
    "ant": ([128, 64], [64, 64]),
    "humanoid": ([256, 128], [128, 128]),
    "mtu": ([400, 200], [400, 200]),
}
# the muscle task's observation: 55 skeleton entries, zero padding to 128, then the 152
# activations (280)
OBS_DIM = {"cartpole": 5, "ant": 37, "humanoid": 76, "mtu": 280}
MTU_OBS_PAD = 128


def state_dim(m):
    return m["nq"] + m["nv"] + (m["na"] if m["has_last_action"] else 0) + m.get("n_mtu", 0)


def initial_states(m, n_envs, seed=1):
    """Initial states of ``n_envs`` envs.

    CartPole: cart at 0, pole angle U(-pi, pi), velocities N(0, 0.1) (std).
    Floating-base tasks: root upright at the model's standing height, hinge angles
    q_mean + N(0, 0.1), zero velocities, zero last action, zero muscle activations.
    """
    rng = np.random.default_rng(seed)
    n_s = state_dim(m)
    s = np.zeros((n_envs, n_s))
    nq, nv = m["nq"], m["nv"]
    if m["task"] == "cartpole":
        s[:, 1] = rng.uniform(-np.pi, np.pi, n_envs)
        s[:, nq:nq + nv] = rng.normal(0.0, 0.1, (n_envs, nv))
        return s
    for j in range(m["n_joints"]):
        a = m["qadr"][j]
        if m["jtype"][j] == FREE:
            s[:, a + 2] = m["root_height"]
            s[:, a + 3] = 1.0
        else:
            s[:, a] = m["q_mean"][j] + rng.normal(0.0, 0.1, n_envs)
    return s


def mlp_params(sizes, seed):
    """Layers [(W [out, in], b [out])], every entry U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    out = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        k = 1.0 / np.sqrt(fi)
        W = rng.uniform(-k, k, (fo, fi))
        b = rng.uniform(-k, k, fo)
        out.append((W, b))
    return out


# name -> (task model, envs, frames h, checkpoint interval)
WORKLOADS = {
    "cartpole": dict(model="cartpole", n_envs=16, h=32),
    "ant": dict(model="ant", n_envs=1024, h=32),
    "humanoid": dict(model="humanoid", n_envs=1024, h=32),
    "mtu": dict(model="mtu_humanoid", n_envs=2048, h=32),
}


def workload(name, n_envs=None, seeds=(1, 2, 3)):
    """Model, initial states, actor and critic weights of a named workload."""
    cfg = WORKLOADS[name]
    m = model_by_name(cfg["model"])
    n = cfg["n_envs"] if n_envs is None else n_envs
    task = m["task"]
    hid_a, hid_c = NETS[task]
    od = OBS_DIM[task]
    actor = mlp_params([od] + hid_a + [m["na"]], seeds[1])
    critic = mlp_params([od] + hid_c + [1], seeds[2])
    s0 = initial_states(m, n, seeds[0])
    return dict(model=m, s0=s0, actor=actor, critic=critic, h=cfg["h"], n_envs=n,
                obs_dim=od, gamma=0.99)
