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
