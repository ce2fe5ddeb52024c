"""The stochastic policy a_t ~ N(mu(s_t), sigma) sampled by reparameterisation (Sec. 3.3),
with the draws passed in: GPU window against the FP64 oracle, bitwise agreement of the
launch forms, the sigma -> 0 limit, and the policy-parameter gradient including
dL/dlog_std; plus the policy-parameter gradient of the muscle task, whose excitations use
the squash (tanh(y) + 1) / 2."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads

pytestmark = pytest.mark.gpu


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def cosine(x, y):
    x, y = np.asarray(x, np.float64).ravel(), np.asarray(y, np.float64).ravel()
    return float(x @ y / (np.linalg.norm(x) * np.linalg.norm(y)))


def _draws(W, h, N, seed=11):
    rng = np.random.default_rng(seed)
    na = W["model"]["na"]
    return rng.standard_normal((h, N, na)), rng.uniform(-1.5, -0.5, na)


def _sim(W, N, h, **kw):
    od = W["obs_dim"]
    return P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                 [od] + [w.shape[0] for w, _ in W["critic"]], **kw)


def _run(W, N, h, noise, log_std, want_theta=False, **kw):
    sim = _sim(W, N, h, policy_grad=want_theta, **kw)
    fw = sim.forward(W["s0"][:N], W["actor"], W["critic"], noise=noise, log_std=log_std)
    ad = sim.adjoint(fw, want_theta=want_theta)
    torch.cuda.synchronize()
    f = {k: fw[k].double().cpu().numpy() for k in ("s_h", "obs", "actions", "rewards", "value")}
    a = {k: ad[k].double().cpu().numpy() for k in ("dL_da", "dL_ds0")}
    if want_theta:
        a["theta"] = ad["dL_dtheta_flat"].double().cpu().numpy()
        a["log_std"] = ad["dL_dlog_std"].double().cpu().numpy()
    return f, a


STOCH = [("cartpole", 16, 8, None), ("ant", 8, 4, 16)]


@pytest.mark.parametrize("name,N,h,k", STOCH, ids=[c[0] for c in STOCH])
def test_stochastic_window_matches_oracle(name, N, h, k):
    W = wl.workload(name, N)
    noise, log_std = _draws(W, h, N)
    print(f"[stoch] {name} N={N} h={h}", flush=True)
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=N,
                              want_theta=True, noise=noise, log_std=log_std)
    want_theta = np.concatenate([x.ravel() for pair in ref["dL_dtheta"] for x in pair])
    f, a = _run(W, N, h, noise, log_std, True, ckpt_interval=k, precision="fp64")
    for key in ("s_h", "actions", "rewards", "value"):
        assert relnorm(f[key], ref[key]) < 1e-10, key
    for got, want in ((a["dL_da"], ref["dL_da"]), (a["dL_ds0"], ref["dL_ds0"]), (a["theta"], want_theta),
                      (a["log_std"], ref["dL_dlog_std"])):
        assert relnorm(got, want) < 1e-9
    f, a = _run(W, N, h, noise, log_std, True, ckpt_interval=k, precision="fp32")
    assert relnorm(f["s_h"], ref["s_h"]) < 1e-4
    for got, want in ((a["dL_da"], ref["dL_da"]), (a["dL_ds0"], ref["dL_ds0"]), (a["theta"], want_theta),
                      (a["log_std"], ref["dL_dlog_std"])):
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3


def test_stochastic_paths_bitwise_and_zero_sigma():
    """The draws enter at the frame start of every launch form identically; with
    sigma = exp(-inf) = 0 the window is bitwise the deterministic one."""
    W = wl.workload("humanoid", 64)
    h = 3
    noise, log_std = _draws(W, h, 64)
    print("[stoch] humanoid paths", flush=True)
    f0, a0 = _run(W, 64, h, noise, log_std, ckpt_interval=4)
    for kw in (dict(ckpt_interval=1), dict(path=P.PATH_TAPE), dict(path=P.PATH_PLAIN)):
        f1, a1 = _run(W, 64, h, noise, log_std, **kw)
        for key in ("s_h", "obs", "actions", "rewards", "value"):
            assert np.array_equal(f0[key], f1[key]), (kw, key)
        assert np.array_equal(a0["dL_da"], a1["dL_da"]), kw
        assert np.array_equal(a0["dL_ds0"], a1["dL_ds0"]), kw
    fz, az = _run(W, 64, h, noise, np.full(W["model"]["na"], -np.inf), ckpt_interval=4)
    sim = _sim(W, 64, h, ckpt_interval=4)
    fd = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fd)
    torch.cuda.synchronize()
    assert np.array_equal(fz["actions"], fd["actions"].double().cpu().numpy())
    assert np.array_equal(fz["s_h"], fd["s_h"].double().cpu().numpy())
    assert np.array_equal(az["dL_da"], ad["dL_da"].double().cpu().numpy())
    assert not np.array_equal(f0["actions"], fz["actions"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_muscle_policy_gradient_matches_oracle(precision):
    W = wl.workload("mtu", 2)
    h = 2
    print(f"[stoch] muscle humanoid policy gradient {precision}", flush=True)
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=2, want_theta=True)
    want = np.concatenate([x.ravel() for pair in ref["dL_dtheta"] for x in pair])
    sim = _sim(W, 2, h, ckpt_interval=16, precision=precision, policy_grad=True)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw, want_theta=True)
    torch.cuda.synchronize()
    got = ad["dL_dtheta_flat"].double().cpu().numpy()
    if precision == "fp64":
        assert relnorm(got, want) < 1e-8
    else:
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3
