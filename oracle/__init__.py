"""FP64 CPU oracle of the differentiable articulated-body window (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, double-precision restatement of what the window
computes, written from the paper's method section and appendix:

* the simulator as a map s_{t+1} = F(s_t, a_t) whose backward pass is the
  vector-Jacobian product of the simulator (Sec. 3.1, Eq. "backward");
* forward dynamics M qdd = J^T f + c + tau (Sec. 3.1, Eq. "fwd_dynamics") with the
  mass matrix and bias written in their defining form (sum over bodies of
  J_b^T I_b J_b and of J_b^T times the Newton-Euler force of body b), solved by a
  Cholesky factorisation and integrated by semi-implicit Euler (Sec. 3.1);
* penalty contact with the linear-step friction law and the joint-limit penalty
  (Sec. 3.1, contact and limit equations);
* the deterministic MLP policy, the task observations and rewards (App. A.3), and
  the short-horizon actor loss (Sec. 3.3, Eq. "policy_loss"; App. A.1);
* the reverse pass is PyTorch reverse-mode differentiation of that forward, which
  is, by construction, the exact adjoint recursion of App. A.1.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path never calls it.
"""
from .dynamics import (OracleModel, substep, dynamics_terms, kinetic_energy, potential_energy,
                       muscle_terms, activation_step)
from .window import (oracle_window, oracle_window_grads, obs_fn, reward_fn, mlp_forward,
                     mlp_forward_bf16, bf16_round, squash, normalize_obs)

__all__ = ["OracleModel", "substep", "dynamics_terms", "kinetic_energy", "potential_energy",
           "oracle_window", "oracle_window_grads", "obs_fn", "reward_fn", "mlp_forward", "normalize_obs"]
