"""FP64 window forward and reverse of the short-horizon actor loss (oracle; tests only).

Forward, per frame t (Sec. 3.3; App. A.3):
    o_t = obs(s_t);  a_t = tanh(MLP_theta(o_t))  (deterministic policy; or given actions)
    r_t = R(s_t, a_t)
    S substeps of the simulator with a_t held;  s_{t+1} = (q, qd[, a_t])
Loss (Sec. 3.3, Eq. "policy_loss"):
    L = -1/(N h) * sum_i [ sum_t gamma^t r_t + gamma^h V(o_h) ]
Reverse (App. A.1): dL/da_t is the adjoint of the action node (the partial of the
appendix's action equation, including the path through the last-action entry of
s_{t+1}), dL/ds_0 is the total derivative through the closed-loop policy, and
dL/dtheta sums (dL/da_t)(d pi / d theta) over envs and frames; all three are
obtained here by reverse-mode differentiation of the forward.
"""
import numpy as np
import torch

from .dynamics import F64, OracleModel, quat_to_rot, substep


def _t(x):
    return torch.as_tensor(np.asarray(x), dtype=F64)


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 the way an FP32 pipeline does: to
    float32 (round to nearest even), then the float32 bit pattern to its top 16 bits
    with round to nearest even (IEEE 754 bfloat16, finite values)."""
    f = x.to(torch.float32).contiguous()
    bits = f.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) >> 16) << 16
    r = torch.where(r >= 2 ** 31, r - 2 ** 32, r).to(torch.int32)
    return r.view(torch.float32).to(F64)


class _BF16Linear(torch.autograd.Function):
    """y = bf16(x) bf16(W)^T + b with exact accumulation; its input adjoint is
    bf16(dy) bf16(W) (the output adjoint enters the transposed product in BF16 as
    well), the weight adjoint dy^T bf16(x)."""

    @staticmethod
    def forward(ctx, x, W, b):
        xr, Wr = bf16_round(x), bf16_round(W)
        ctx.save_for_backward(xr, Wr)
        return xr @ Wr.T + b

    @staticmethod
    def backward(ctx, gy):
        xr, Wr = ctx.saved_tensors
        return bf16_round(gy) @ Wr, gy.T @ xr, gy.sum(0)


def mlp_forward_bf16(layers, x):
    """The MLP with BF16 weights and BF16 layer inputs and exact (float64) accumulation
    of their products: the reference of the BF16 matrix-core MLPs (FP32 biases and
    activations)."""
    h = x
    for i, (W, b) in enumerate(layers):
        h = _BF16Linear.apply(h, W, b)
        if i < len(layers) - 1:
            h = torch.nn.functional.elu(h)
    return h


def layer_norm(a, g, b, eps):
    """Layer normalisation of each row of a (Ba, Kiros and Hinton): the row's mean and
    population variance, a_hat = (a - mean) / sqrt(var + eps), then the gain and bias,
    g * a_hat + b."""
    mu = a.mean(-1, keepdim=True)
    var = ((a - mu) ** 2).mean(-1, keepdim=True)
    return g * ((a - mu) / torch.sqrt(var + eps)) + b


def mlp_forward(layers, x, ln=None, ln_eps=1e-5):
    """ELU hidden layers, linear output (App. A.2 network description).  ln: None (no
    normalisation), or per hidden layer the (gain, bias) of a layer normalisation applied to
    that layer's ELU output (App. A.2: layer normalisation on each hidden layer)."""
    h = x
    n = len(layers)
    for i, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if i < n - 1:
            h = torch.where(h > 0, h, torch.expm1(torch.clamp(h, max=0.0)))
            if ln is not None:
                g, beta = ln[i]
                h = layer_norm(h, g, beta, ln_eps)
    return h


def obs_fn(m, s):
    """Observation vector of the task (App. A.3 observation tables)."""
    task = m.md["task"]
    nq, nv = m.nq, m.nv
    q, qd = s[:, :nq], s[:, nq:nq + nv]
    if task == "none":
        return s                              # no task: the state itself
    if task == "cartpole":
        x, th, xd, thd = q[:, 0], q[:, 1], qd[:, 0], qd[:, 1]
        return torch.stack([x, xd, torch.sin(th), torch.cos(th), thd], 1)
    R = quat_to_rot(q[:, 3:7])
    up = R[:, 2, 2]
    heading = R[:, 0, 0]
    parts = [q[:, 2:3], q[:, 3:7], qd[:, 0:3], qd[:, 3:6], q[:, 7:], qd[:, 6:],
             up[:, None], heading[:, None]]
    if m.md["has_last_action"]:
        parts.append(s[:, nq + nv:nq + nv + m.na])
    if task == "mtu":
        # skeleton observation, zero padding to 128 entries, then the activations
        sk = torch.cat(parts, 1)
        pad = torch.zeros(s.shape[0], 128 - sk.shape[1], dtype=F64)
        return torch.cat([sk, pad, s[:, nq + nv:nq + nv + m.n_mtu]], 1)
    return torch.cat(parts, 1)


def reward_fn(m, s, a):
    """Single-step reward R(s_t, a_t) (App. A.3 reward definitions)."""
    task = m.md["task"]
    nq, nv = m.nq, m.nv
    q, qd = s[:, :nq], s[:, nq:nq + nv]
    if task == "none":
        return torch.zeros(s.shape[0], dtype=F64)
    if task == "cartpole":
        th = torch.atan2(torch.sin(q[:, 1]), torch.cos(q[:, 1]))
        return -th ** 2 - 0.1 * qd[:, 1] ** 2 - 0.05 * q[:, 0] ** 2 - 0.1 * qd[:, 0] ** 2
    R = quat_to_rot(q[:, 3:7])
    up, heading, hgt, vx = R[:, 2, 2], R[:, 0, 0], q[:, 2], qd[:, 0]
    if task == "ant":
        return vx + 0.1 * up + heading + (hgt - 0.27)
    if task == "humanoid":
        dh = torch.clamp(hgt - 0.84, -1.0, 0.1)
        rh = torch.where(dh < 0, -200.0 * dh * dh, 10.0 * dh)
        return vx + 0.1 * up + heading + rh - 0.002 * (a * a).sum(1)
    if task == "mtu":
        # App. A.3 muscle-task reward, at the humanoid skeleton's torso height reference
        dh = torch.clamp(hgt - 0.84, -1.0, 0.05)
        rh = torch.where(dh < 0, -200.0 * dh * dh, 4.0 * dh)
        return vx + 0.1 * up + heading + rh - 0.001 * (a * a).sum(1)
    raise ValueError(task)


def squash(m, y):
    """Policy output to action: tanh for torques, (tanh + 1)/2 for muscle excitations."""
    if m.md["task"] == "mtu":
        return 0.5 * (torch.tanh(y) + 1.0)
    return torch.tanh(y)


def _layers(params):
    return [(_t(W), _t(b)) for (W, b) in params]


def _ln(params):
    return None if params is None else [(_t(g), _t(b)) for (g, b) in params]


def fp32_round(x):
    """Each entry rounded to the nearest float32 value (round to nearest even), kept in
    float64.  The derivative is taken as the identity (straight through), so that the
    reverse pass of a rounded window is the FP64 adjoint along the rounded trajectory."""
    r = x.detach().to(torch.float32).to(F64)
    return x + (r - x).detach()


def normalize_obs(o, obs_norm):
    """Observation normalisation with running statistics (Sec. 3.3): the networks read
    (o - mean) * inv_std; obs_norm = (mean, inv_std), or None for the raw observation."""
    if obs_norm is None:
        return o
    mean, inv_std = (x if torch.is_tensor(x) else _t(x) for x in obs_norm)
    return (o - mean) * inv_std


def oracle_window(md, s0, h, actor=None, critic=None, actions=None, gamma=0.99, n_total=None,
                  keep_graph=False, layers=None, action_offset=None, bf16=False, noise=None, log_std=None,
                  reset_states=None, obs_norm=None, diagnostics=True, fp32_floor=False, actor_ln=None,
                  critic_ln=None, ln_eps=1e-5):
    """Run one window.  Returns a dict of float64 tensors (numpy on request by caller).

    s0: [B, n_s]; actions (open loop) [h, B, na] or None (closed loop through ``actor``).
    n_total: the N of the 1/(N h) loss scale (defaults to B).
    action_offset: optional [h, B, na] added to each action (used by finite-difference
    checks of dL/da_t).
    bf16: evaluate actor and critic with BF16 weights and layer inputs (mlp_forward_bf16).
    noise [h, B, na], log_std [na]: the stochastic policy a_t ~ N(mu(s_t), sigma) sampled by
    reparameterisation (Sec. 3.3): the pre-squash output is mu(o_t) + exp(log_std) noise_t.
    reset_states [B, n_s]: early termination (App. A.3) for a model with "term_height": an env
    whose root is below that height at the end of a frame restarts from its reset state (a
    constant), and its discount restarts at the next frame; a segment that ends in a
    termination has no terminal value.
    obs_norm = (mean, inv_std) [od]: actor and critic read normalised observations; the
    returned obs stay raw.
    diagnostics: also count, per env, the contact evaluations whose normal force pulls
    ("adhesive"); off when only the method's own arithmetic should run.
    fp32_floor: the FP32 storage floor.  The initial states and the network weights are
    rounded to float32 on entry, every action when it is formed, and the dynamic state
    (q, qd and the muscle activations) after every substep; all arithmetic stays FP64.  It
    measures how far the window alone carries the rounding of the state that any FP32
    simulator stores (the intrinsic sensitivity floor of an FP32 window).  Off, nothing
    changes.
    actor_ln / critic_ln: per hidden layer the (gain, bias) of the layer normalisation of the
    actor's / critic's hidden layers (App. A.2), or None; ln_eps its variance offset.
    The result holds the loss and, in loss_env [B], each env's term of it.
    """
    m = md if isinstance(md, OracleModel) else OracleModel(md)
    s = s0 if torch.is_tensor(s0) else _t(s0)
    B = s.shape[0]
    N = B if n_total is None else n_total
    if layers is None:
        layers = (_layers(actor) if actor is not None else None,
                  _layers(critic) if critic is not None else None)
    act_l, crit_l = layers
    a_ln = actor_ln if actor_ln is None or torch.is_tensor(actor_ln[0][0]) else _ln(actor_ln)
    c_ln = critic_ln if critic_ln is None or torch.is_tensor(critic_ln[0][0]) else _ln(critic_ln)
    if fp32_floor:
        s = fp32_round(s)
        act_l = [(fp32_round(W), fp32_round(b)) for (W, b) in act_l] if act_l is not None else None
        crit_l = [(fp32_round(W), fp32_round(b)) for (W, b) in crit_l] if crit_l is not None else None
    rnd = fp32_round if fp32_floor else (lambda x: x)
    nq, nv = m.nq, m.nv
    dt = m.dt / m.substeps
    if bf16:
        if a_ln is not None or c_ln is not None:
            raise ValueError("layer normalisation is not modelled with BF16 networks")
        mlp = lambda lay, x, ln=None: mlp_forward_bf16(lay, x)
    else:
        mlp = lambda lay, x, ln=None: mlp_forward(lay, x, ln, ln_eps)
    states, obs, acts, rews = [s], [], [], []
    term_h = m.md.get("term_height") if reset_states is not None else None
    t0 = torch.zeros(B, dtype=torch.long)
    segs, dones = [], []
    adh = [] if diagnostics else None
    for t in range(h):
        o = obs_fn(m, s)
        if actions is None:
            y = mlp(act_l, normalize_obs(o, obs_norm), a_ln)
            if noise is not None:
                ls = log_std if torch.is_tensor(log_std) else _t(log_std)
                y = y + torch.exp(ls) * (noise[t] if torch.is_tensor(noise) else _t(noise[t]))
            a = squash(m, y)
        else:
            a = actions[t] if torch.is_tensor(actions[t]) else _t(actions[t])
        a = rnd(a)
        if action_offset is not None:
            a = a + _t(action_offset[t])
        if keep_graph and not a.requires_grad:
            a.requires_grad_(True)
        r = reward_fn(m, s, a)
        q, qd = s[:, :nq], s[:, nq:nq + nv]
        if m.n_mtu:
            act = s[:, nq + nv:nq + nv + m.n_mtu]
            for _ in range(m.substeps):
                q, qd, act = substep(m, q, qd, a, dt, act, stats=adh)
                q, qd, act = rnd(q), rnd(qd), rnd(act)
            s = torch.cat([q, qd, act], 1)
        else:
            for _ in range(m.substeps):
                q, qd = substep(m, q, qd, a, dt, stats=adh)
                q, qd = rnd(q), rnd(qd)
            s = torch.cat([q, qd, a], 1) if m.md["has_last_action"] else torch.cat([q, qd], 1)
        if term_h is not None:
            done = s[:, 2] < term_h
            s = torch.where(done[:, None], _t(reset_states), s)
            segs.append(t0.clone())
            dones.append(done)
            t0 = torch.where(done, torch.full_like(t0, t + 1), t0)
        states.append(s)
        obs.append(o)
        acts.append(a)
        rews.append(r)
    o_h = obs_fn(m, s)
    obs.append(o_h)
    value = mlp(crit_l, normalize_obs(o_h, obs_norm), c_ln)[:, 0] if crit_l is not None else torch.zeros(B, dtype=F64)
    if term_h is None:
        disc = sum(gamma ** t * rews[t] for t in range(h))
        loss = -(disc + gamma ** h * value).sum() / (N * h)
        loss_env = -(disc + gamma ** h * value) / (N * h)
        done_out = None
    else:
        disc = sum(torch.pow(gamma, (t - segs[t]).to(F64)) * rews[t] for t in range(h))
        live = (~dones[-1]).to(F64)
        loss = -(disc + live * torch.pow(gamma, (h - t0).to(F64)) * value).sum() / (N * h)
        loss_env = -(disc + live * torch.pow(gamma, (h - t0).to(F64)) * value) / (N * h)
        done_out = torch.stack(dones)
    adhesive = torch.stack(adh).sum(0) if adh else torch.zeros(B, dtype=torch.long)
    return dict(states=states, obs=obs, actions=acts, rewards=rews, value=value, loss=loss,
                loss_env=loss_env, layers=layers, done=done_out, adhesive=adhesive)


def oracle_window_grads(md, s0, h, actor=None, critic=None, actions=None, gamma=0.99,
                        n_total=None, want_theta=False, bf16=False, noise=None, log_std=None,
                        reset_states=None, obs_norm=None, fp32_floor=False, actor_ln=None, critic_ln=None,
                        ln_eps=1e-5):
    """Window forward plus its exact reverse (App. A.1) by reverse-mode differentiation.
    fp32_floor: as for oracle_window (the FP32 storage floor); the gradients are then the
    FP64 adjoint along the rounded trajectory.
    actor_ln / critic_ln, ln_eps: as for oracle_window; with want_theta the result also holds
    dL_dln, the (gain, bias) gradients of the actor's layer normalisations.

    Returns numpy arrays: s_h, obs [h+1,B,od], actions [h,B,na], rewards [h,B],
    value [B], loss, dL/da [h,B,na], dL/ds0 [B,n_s] and, if asked, dL/dtheta as a
    list of (dW, db) per actor layer.
    """
    s0t = _t(s0).clone().requires_grad_(True)
    layers = None
    if actor is not None:
        layers = ([(W.clone().requires_grad_(want_theta), b.clone().requires_grad_(want_theta))
                   for (W, b) in _layers(actor)],
                  _layers(critic) if critic is not None else None)
    act_in = None
    if actions is not None:
        act_in = [_t(actions[t]).clone().requires_grad_(True) for t in range(h)]
    ls = None
    if noise is not None:
        ls = _t(log_std).clone().requires_grad_(want_theta)
    a_ln = None
    if actor_ln is not None:
        a_ln = [(_t(g).clone().requires_grad_(want_theta), _t(b).clone().requires_grad_(want_theta))
                for (g, b) in actor_ln]
    out = oracle_window(md, s0t, h, actor, critic, act_in, gamma, n_total, keep_graph=True,
                        layers=layers, bf16=bf16, noise=noise, log_std=ls, reset_states=reset_states,
                        obs_norm=obs_norm, fp32_floor=fp32_floor, actor_ln=a_ln, critic_ln=critic_ln,
                        ln_eps=ln_eps)
    wrt = [s0t] + list(out["actions"])
    theta = []
    if want_theta and actor is not None:
        for (W, b) in layers[0]:
            theta += [W, b]
        if a_ln is not None:
            for (g, b) in a_ln:
                theta += [g, b]
        if ls is not None:
            theta.append(ls)
    g = torch.autograd.grad(out["loss"], wrt + theta, allow_unused=True)
    gs0 = g[0]
    ga = torch.stack([x if x is not None else torch.zeros_like(out["actions"][0])
                      for x in g[1:1 + h]])
    res = dict(
        s_h=out["states"][-1].detach().numpy(),
        states=torch.stack(out["states"]).detach().numpy(),
        obs=torch.stack(out["obs"]).detach().numpy(),
        actions=torch.stack(out["actions"]).detach().numpy(),
        rewards=torch.stack(out["rewards"]).detach().numpy(),
        value=out["value"].detach().numpy(),
        loss=float(out["loss"].detach()),
        loss_env=out["loss_env"].detach().numpy(),
        dL_da=ga.detach().numpy(),
        dL_ds0=gs0.detach().numpy(),
    )
    res["adhesive"] = out["adhesive"].numpy()
    if out["done"] is not None:
        res["done"] = out["done"].numpy()
    if want_theta and actor is not None:
        gt = g[1 + h:]
        if ls is not None:
            res["dL_dlog_std"] = gt[-1].numpy()
            gt = gt[:-1]
        nl = len(layers[0])
        res["dL_dtheta"] = [(gt[2 * i].numpy(), gt[2 * i + 1].numpy()) for i in range(nl)]
        if a_ln is not None:
            res["dL_dln"] = [(gt[2 * nl + 2 * i].numpy(), gt[2 * nl + 2 * i + 1].numpy())
                             for i in range(len(a_ln))]
    return res
