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


if __name__ == "__main__":
    print(count_env_step())
