"""The oracle's operation counter: pinned to textbook operation counts, and the counted
humanoid env-step that the benchmark quotes."""
import os
import sys

import torch

from oracle.count_ops import OpCounter, count_env_step

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_counter_textbook_counts():
    a = torch.rand(3, 4, dtype=torch.float64)
    b = torch.rand(4, 5, dtype=torch.float64)
    with OpCounter() as c:
        a @ b                                           # 2 m n k
    assert c.flops == 2 * 3 * 5 * 4
    x = torch.rand(7, 6, dtype=torch.float64)
    with OpCounter() as c:
        (x * x + x).sum()                               # 42 + 42 + 42
    assert c.flops == 3 * 42
    A = torch.rand(27, 27, dtype=torch.float64)
    M = A @ A.T + 27.0 * torch.eye(27, dtype=torch.float64)
    with OpCounter() as c:
        L = torch.linalg.cholesky(M)                    # n^3 / 3
    assert c.flops == 27 ** 3 // 3
    rhs = torch.rand(27, 2, dtype=torch.float64)
    with OpCounter() as c:
        torch.cholesky_solve(rhs, L)                    # two triangular solves per column
    assert c.flops == 2 * 2 * 27 * 27
    with OpCounter() as c:
        torch.zeros(5).clone().reshape(5, 1)            # data movement counts zero
    assert c.flops == 0 and not c.uncounted


def test_humanoid_env_step_count_matches_bench():
    import bench
    got = count_env_step("humanoid")
    assert not got["uncounted_ops"], got["uncounted_ops"]
    assert got["forward"] == bench.ORACLE_OPS_PER_ENV_STEP["forward"]
    assert got["reverse"] == bench.ORACLE_OPS_PER_ENV_STEP["reverse"]


def test_recursive_substep_counts_match_bench():
    """The algorithmic operation counts of one humanoid substep (recursive algorithms) and of
    its implicit-function adjoint, and of the per-frame work around the substeps, that the
    benchmark's roofline uses."""
    import bench
    from oracle.count_ops import count_frame_level, count_recursive_substep
    sub = count_recursive_substep("humanoid")
    fr = count_frame_level("humanoid")
    assert not sub["uncounted_ops"] and not fr["uncounted_ops"]
    assert (sub["forward"], sub["reverse"]) == (bench.ALGO_OPS["substep_forward"], bench.ALGO_OPS["substep_reverse"])
    assert (fr["forward"], fr["reverse"]) == (bench.ALGO_OPS["frame_forward"], bench.ALGO_OPS["frame_reverse"])


def test_recursive_counts_scale_like_the_textbook():
    """The counts grow as the algorithms do: the Cholesky factorisation's n^3 / 3 and the two
    solves' 2 n^2 are inside the forward count, and the substep costs more with more bodies,
    DOFs and contacts (CartPole < Ant < Humanoid)."""
    from oracle.count_ops import count_recursive_substep
    c = {n: count_recursive_substep(n) for n in ("cartpole", "ant", "humanoid")}
    assert c["cartpole"]["forward"] < c["ant"]["forward"] < c["humanoid"]["forward"]
    assert c["cartpole"]["reverse"] < c["ant"]["reverse"] < c["humanoid"]["reverse"]
    n = c["humanoid"]["nv"]
    assert c["humanoid"]["forward"] > n ** 3 // 3 + 2 * n * n
