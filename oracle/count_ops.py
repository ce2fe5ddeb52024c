"""Floating-point operation count of the FP64 oracle (TEST INFRASTRUCTURE ONLY).

Every tensor operation the oracle performs, in its forward window and in the
reverse-mode pass that gives dL/da and dL/ds0, is intercepted at the dispatcher and
counted: one operation per output element for element-wise arithmetic (two for fused
multiply-add forms), 2 m n k for a matrix product, one per input element for a
reduction, n^3 / 3 for a Cholesky factorisation and 2 n^2 per right-hand side for a
triangular solve.  Data movement (views, copies, concatenation, indexing, selection,
comparisons) counts zero.  The oracle has no data-dependent control flow, so the count
depends only on the model and the network shapes.

The oracle computes the mass matrix and the bias in their defining dense form (sums of
J^T I J and J^T f over bodies), so its count is larger than that of the recursive
algorithm the GPU kernels run; it is a property of the reference computation, not a
roofline figure for the kernels.

    python -m oracle.count_ops        # prints the per-env-step counts of the humanoid
"""
import collections

import torch
from torch.utils._python_dispatch import TorchDispatchMode

from .window import oracle_window

_ELEMENTWISE_1 = {
    "add", "sub", "mul", "div", "neg", "sqrt", "rsqrt", "reciprocal", "sin", "cos", "exp",
    "expm1", "tanh", "pow", "abs", "clamp", "clamp_min", "clamp_max", "maximum", "minimum",
    "rsub", "sgn", "sign", "square", "elu", "threshold_backward", "log", "atan2", "acos",
}
_ELEMENTWISE_2 = {"addcmul", "addcdiv", "lerp", "tanh_backward", "elu_backward", "sigmoid_backward"}
_REDUCTIONS = {"sum", "mean", "prod", "amax", "amin", "cumsum", "linalg_vector_norm", "norm", "dot", "vdot"}
_ZERO = {
    "view", "_unsafe_view", "reshape", "expand", "permute", "transpose", "t", "squeeze", "unsqueeze",
    "select", "slice", "cat", "stack", "clone", "copy", "copy_", "_to_copy", "detach", "alias",
    "zeros", "zeros_like", "ones_like", "empty", "empty_like", "new_zeros", "new_empty", "new_ones",
    "fill", "fill_", "zero_", "full", "full_like", "eye", "lift_fresh", "index", "index_put",
    "index_put_", "gather", "scatter", "scatter_add", "index_select", "where", "lt", "le", "gt", "ge",
    "eq", "ne", "logical_not", "logical_and", "logical_or", "masked_fill", "as_strided", "split",
    "split_with_sizes", "unbind", "diag_embed", "diagonal", "diag", "tril", "triu", "narrow",
    "contiguous", "ones", "scalar_tensor", "_local_scalar_dense", "arange", "sum_to_size",
    "slice_backward", "select_backward", "expand_copy", "_conj", "conj", "resolve_conj", "resolve_neg",
    "_reshape_alias", "new_full", "masked_fill_", "flip", "roll", "repeat", "unsqueeze_copy",
    "squeeze_copy", "view_copy", "permute_copy", "transpose_copy", "t_copy", "clone_", "is_same_size",
    "_index_put_impl_", "diagonal_backward", "diagonal_scatter", "slice_scatter", "select_scatter",
    "_linalg_check_errors",
}


class OpCounter(TorchDispatchMode):
    """Counts floating-point operations of the tensor operations run under it."""

    def __init__(self):
        super().__init__()
        self.flops = 0
        self.by_op = collections.Counter()
        self.uncounted = collections.Counter()

    def _add(self, name, n):
        self.flops += int(n)
        self.by_op[name] += int(n)

    def __torch_dispatch__(self, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        out = func(*args, **kwargs)
        name = func.overloadpacket.__name__.rstrip("_")
        o = out[0] if isinstance(out, (tuple, list)) else out
        numel = o.numel() if torch.is_tensor(o) else 0
        if name in ("mm", "bmm", "addmm", "baddbmm", "addbmm"):
            a = args[1] if name in ("addmm", "baddbmm", "addbmm") else args[0]
            k = a.shape[-1]
            self._add(name, 2 * numel * k + (numel if name.startswith("add") or name == "baddbmm" else 0))
        elif name == "mv":
            self._add(name, 2 * args[0].numel())
        elif name in ("linalg_cholesky_ex", "cholesky"):
            n = args[0].shape[-1]
            self._add(name, args[0].numel() // (n * n) * (n ** 3) // 3)
        elif name == "cholesky_solve":
            b, L = args[0], args[1]
            n = L.shape[-1]
            self._add(name, (b.numel() // n) * 2 * 2 * n * n // 2)
        elif name in ("linalg_solve_triangular", "triangular_solve"):
            A, B = (args[0], args[1]) if name == "linalg_solve_triangular" else (args[1], args[0])
            n = A.shape[-1]
            self._add(name, (B.numel() // n) * n * n)
        elif name == "linalg_cross":
            self._add(name, 2 * numel)
        elif name in _ELEMENTWISE_1:
            self._add(name, numel)
        elif name in _ELEMENTWISE_2:
            self._add(name, 2 * numel)
        elif name in _REDUCTIONS:
            self._add(name, sum(x.numel() for x in args if torch.is_tensor(x)))
        elif name not in _ZERO:
            self.uncounted[name] += 1
        return out


def count_window(md, s0, h, actor, critic):
    """(forward, reverse, counter objects) of one window of the given envs."""
    s0t = torch.as_tensor(s0, dtype=torch.float64).clone().requires_grad_(True)
    cf = OpCounter()
    with cf:
        out = oracle_window(md, s0t, h, actor, critic, keep_graph=True, diagnostics=False)
    cr = OpCounter()
    with cr:
        torch.autograd.grad(out["loss"], [s0t] + list(out["actions"]))
    return cf.flops, cr.flops, cf, cr


def count_env_step(name="humanoid"):
    """Operations of one env-step (one frame of one env): the difference of windows of two
    and one frames, so the terminal critic and its reverse drop out."""
    import workloads as wl
    W = wl.workload(name, 1)
    f1, r1, _, _ = count_window(W["model"], W["s0"], 1, W["actor"], W["critic"])
    f2, r2, cf, cr = count_window(W["model"], W["s0"], 2, W["actor"], W["critic"])
    return {"forward": f2 - f1, "reverse": r2 - r1, "substeps": int(W["model"]["substeps"]),
            "uncounted_ops": sorted(set(cf.uncounted) | set(cr.uncounted))}


def count_recursive_substep(name="humanoid"):
    """Algorithmic operations of one substep of the recursive algorithms (``recursive``) and
    of its adjoint by the implicit-function theorem, counted on one env.

    forward: kinematics, velocities, contact forces, recursive Newton-Euler bias, composite-
    rigid-body mass matrix, Cholesky factorisation and solve, semi-implicit Euler.
    reverse: the integrator's reverse, lambda = M^{-1} q_ddot_bar by the two triangular solves
    of the cached factor, inverse dynamics at the solved q_ddot on the forward's kinematics
    (the accelerations and Newton-Euler forces the derivative needs), and its vector-Jacobian
    product with lambda with respect to (q, q_dot, a) through kinematics, contacts, limits and
    actuation.  Re-running the forward (recomputation from a checkpoint) is not counted: it is a
    memory trade-off, not part of the algorithm."""
    import workloads as wl
    from .dynamics import OracleModel, integrate, joint_torques
    from .recursive import inverse_dynamics, kinematics, substep_recursive
    W = wl.workload(name, 1)
    m = OracleModel(W["model"])
    dt = m.dt / m.substeps
    s = torch.as_tensor(W["s0"], dtype=torch.float64)
    q0, qd0 = s[:, :m.nq].clone(), s[:, m.nq:m.nq + m.nv].clone()
    a0 = torch.full((1, m.na), 0.3, dtype=torch.float64)
    with OpCounter() as cf:
        substep_recursive(m, q0, qd0, a0, dt)
    q = q0.clone().requires_grad_(True)
    qd = qd0.clone().requires_grad_(True)
    a = a0.clone().requires_grad_(True)
    with torch.no_grad():
        _, qd_new0, qdd0, L = substep_recursive(m, q0, qd0, a0, dt)
    qd_new = qd_new0.clone().requires_grad_(True)
    q_new = integrate(m, q, qd_new, dt)
    kin = kinematics(m, q, qd)
    gq, gqd = torch.ones_like(q_new), torch.ones_like(qd_new)
    cr = OpCounter()
    with cr:
        # integrator: q' = integrate(q, qd'), qd' = qd + dt qdd
        bq, bqdn = torch.autograd.grad(q_new, [q, qd_new], gq, retain_graph=True)
        bqdn = bqdn + gqd
        qddbar = dt * bqdn
        lam = torch.cholesky_solve(qddbar[..., None], L)[..., 0]
        ID = inverse_dynamics(m, q, qd, qdd0, kin=kin) - joint_torques(m, q, a)
        gq_id, gqd_id, _ = torch.autograd.grad(ID, [q, qd, a], -lam)
        bq + gq_id, bqdn + gqd_id                    # the adjoints of the pre-substep state
    return {"forward": cf.flops, "reverse": cr.flops, "nv": m.nv,
            "uncounted_ops": sorted(set(cf.uncounted) | set(cr.uncounted))}


def count_frame_level(name="humanoid"):
    """Operations of the per-frame work of one env around the substeps: observation, actor
    MLP, squash and reward (forward), and their reverse: the reward's and the observation's
    vector-Jacobian products and the actor's input VJP (the policy feedback of App. A.1)."""
    import workloads as wl
    from .dynamics import OracleModel
    from .window import _layers, mlp_forward, obs_fn, reward_fn, squash
    W = wl.workload(name, 1)
    m = OracleModel(W["model"])
    s = torch.as_tensor(W["s0"], dtype=torch.float64).clone().requires_grad_(True)
    act = _layers(W["actor"])
    with OpCounter() as cf:
        o = obs_fn(m, s)
        a = squash(m, mlp_forward(act, o))
        r = reward_fn(m, s, a)
    with OpCounter() as cr:
        torch.autograd.grad(r.sum() + (a * torch.ones_like(a)).sum(), [s])
    return {"forward": cf.flops, "reverse": cr.flops,
            "uncounted_ops": sorted(set(cf.uncounted) | set(cr.uncounted))}


if __name__ == "__main__":
    print(count_env_step())
    print(count_recursive_substep())
    print(count_frame_level())
