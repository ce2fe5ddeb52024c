"""The factor cache of the persistent path (Sec. 3.1: the factorisation cached for the backward
pass): the forward keeps every substep's Cholesky factor, reciprocal pivots and accelerations,
and the adjoint rebuilds each checkpoint segment's states from the accelerations and recomputes
only the kinematics, contacts and body inertias.  The arithmetic of every value the adjoint
reads is the forward's own, so the window's outputs and gradients must equal, bit for bit,
those of the other launch forms; the FP64 instantiation is also held to the oracle."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads

pytestmark = pytest.mark.gpu

FWD_KEYS = ("s_h", "obs", "actions", "rewards", "value")


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def _dims(W):
    od = W["obs_dim"]
    return [od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]]


def _run(W, md, N, h, s0=None, want_theta=False, fw_kw=None, **kw):
    ad_, cd_ = _dims(W)
    sim = P.Sim(md, N, h, ad_, cd_, policy_grad=want_theta, **kw)
    fw = sim.forward(W["s0"][:N] if s0 is None else s0, W["actor"], W["critic"], **(fw_kw or {}))
    ad = sim.adjoint(fw, want_theta=want_theta)
    torch.cuda.synchronize()
    f = {k: v.double().cpu().numpy() for k, v in fw.items() if torch.is_tensor(v)}
    a = {k: v.double().cpu().numpy() for k, v in ad.items() if torch.is_tensor(v)}
    sim.close()
    return f, a


def _same(ref, got, keys):
    for key in keys:
        assert np.array_equal(ref[key], got[key]), key


@pytest.mark.parametrize("name,k", [("cartpole", 4), ("ant", 4), ("humanoid", 4), ("humanoid", 16), ("humanoid", 1)])
def test_factor_cache_bitwise_equal_to_recompute_and_tape(name, k):
    W = wl.workload(name, 64)
    md, h = W["model"], 3
    print(f"[factor cache] {name} k={k}: cached / recomputed / tape", flush=True)
    f0, a0 = _run(W, md, 64, h, want_theta=True, ckpt_interval=k, factor_cache=True)
    for kw in (dict(ckpt_interval=k), dict(path=P.PATH_TAPE)):
        f1, a1 = _run(W, md, 64, h, want_theta=True, **kw)
        _same(f0, f1, FWD_KEYS)
        _same(a0, a1, ("dL_da", "dL_ds0", "dL_dtheta_flat"))


def test_factor_cache_fp64_full_window_matches_oracle():
    """FP64 kernels with the factor cache over the full Ant window (N 256, k 4) against the
    oracle on sampled envs (the bar of the tape path's FP64 test)."""
    W = wl.workload("ant", 256)
    h = W["h"]
    print("[factor cache] ant 256 fp64 full window vs oracle", flush=True)
    f, a = _run(W, W["model"], 256, h, ckpt_interval=4, factor_cache=True, precision="fp64")
    envs = [7, 200]
    ref = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], n_total=256)
    assert relnorm(f["s_h"][envs], ref["s_h"]) < 1e-9
    assert relnorm(a["dL_da"][:, envs], ref["dL_da"]) < 1e-9
    assert relnorm(a["dL_ds0"][envs], ref["dL_ds0"]) < 1e-9


def test_factor_cache_with_forced_fp64_fallback():
    """Every substep refactorised in FP64 (threshold above 1): the cache holds no FP64 factor,
    so the adjoint recomputes each flagged substep whole; the result is bitwise that of the
    persistent path without the cache."""
    W = wl.workload("humanoid", 64)
    h = 2
    print("[factor cache] humanoid forced fallback", flush=True)
    f0, a0 = _run(W, W["model"], 64, h, ckpt_interval=4, factor_cache=True, chol_fp64_threshold=2.0)
    f1, a1 = _run(W, W["model"], 64, h, ckpt_interval=4, chol_fp64_threshold=2.0)
    assert (f0["fp64_refactor_count"] == h * 48).all()
    _same(f0, f1, FWD_KEYS)
    _same(a0, a1, ("dL_da", "dL_ds0"))


@pytest.mark.parametrize("lanes", [0, 32])
def test_factor_cache_with_termination_noise_and_normalisation(lanes):
    """Ant with early termination (a reset every frame), the stochastic policy and observation
    normalisation, in the full layout and in the compact layout: cached against the tape path."""
    W = wl.workload("ant", 64)
    md = wl.with_termination(W["model"])
    s0 = W["s0"].copy()
    s0[::2, 2] = 0.2
    reset = wl.initial_states(md, 64, seed=9)
    reset[::4, 2] = 0.2
    h = 4
    rng = np.random.default_rng(11)
    noise = torch.as_tensor(rng.standard_normal((h, 64, md["na"])), dtype=torch.float32, device="cuda")
    log_std = torch.full((md["na"],), -1.0, dtype=torch.float32, device="cuda")
    mean = torch.as_tensor(rng.normal(size=W["obs_dim"]) * 0.1, dtype=torch.float32, device="cuda")
    inv = torch.as_tensor(rng.uniform(0.5, 2.0, W["obs_dim"]), dtype=torch.float32, device="cuda")
    fw_kw = dict(reset_states=reset, noise=noise, log_std=log_std, obs_norm=(mean, inv))
    print(f"[factor cache] ant termination + noise + normalisation, lanes {lanes}", flush=True)
    f0, a0 = _run(W, md, 64, h, s0=s0, want_theta=True, fw_kw=fw_kw, ckpt_interval=4, factor_cache=True,
                  lanes_per_env=lanes)
    f1, a1 = _run(W, md, 64, h, s0=s0, want_theta=True, fw_kw=fw_kw, path=P.PATH_TAPE)
    assert f0["done"].any()
    _same(f0, f1, FWD_KEYS + ("done", "loss", "loss_env"))
    _same(a0, a1, ("dL_da", "dL_ds0", "dL_dtheta_flat", "dL_dlog_std"))
