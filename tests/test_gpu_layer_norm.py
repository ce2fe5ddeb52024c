"""Layer normalisation of the hidden layers of the actor and the critic (App. A.2: ELU hidden
layers, each followed by a layer normalisation with a gain and a bias), switched on with
SimOptions.layer_norm: the in-kernel MLPs of the window, their input adjoints, the
policy-parameter gradient (which then includes the gains and biases) and the critic values,
against the oracle's layer-normalised MLP (oracle.window.mlp_forward with ln)."""
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


def ln_params(widths, seed):
    """Seeded gains U(0.5, 1.5) and biases N(0, 0.2) of the hidden layers' normalisations."""
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0.5, 1.5, w), rng.normal(0.0, 0.2, w)) for w in widths]


def _case(name, N):
    W = wl.workload(name, N)
    od = W["obs_dim"]
    ad = [od] + [w.shape[0] for w, _ in W["actor"]]
    cd = [od] + [w.shape[0] for w, _ in W["critic"]]
    return W, ad, cd, ln_params(ad[1:-1], 21), ln_params(cd[1:-1], 22)


def _run(W, ad, cd, a_ln, c_ln, N, h, precision, **kw):
    sim = P.Sim(W["model"], N, h, ad, cd, precision=precision, policy_grad=True, layer_norm=True, **kw)
    fw = sim.forward(W["s0"][:N], W["actor"], W["critic"], actor_ln=a_ln, critic_ln=c_ln)
    ad_ = sim.adjoint(fw, want_theta=True)
    torch.cuda.synchronize()
    f = {k: fw[k].double().cpu().numpy() for k in ("s_h", "obs", "actions", "rewards", "value", "loss")}
    a = {k: ad_[k].double().cpu().numpy() for k in ("dL_da", "dL_ds0", "dL_dtheta_flat")}
    return sim, f, a


def _theta_ref(ref):
    """The oracle's actor gradient in the library's flat order: per layer W, b, then the
    layer's normalisation gain and bias (hidden layers)."""
    parts = []
    nl = len(ref["dL_dtheta"])
    for i, (dW, db) in enumerate(ref["dL_dtheta"]):
        parts += [dW.ravel(), db.ravel()]
        if i < nl - 1:
            dg, dbeta = ref["dL_dln"][i]
            parts += [dg.ravel(), dbeta.ravel()]
    return np.concatenate(parts)


@pytest.mark.parametrize("name,N,h,tol", [("cartpole", 16, 32, 1e-10), ("ant", 8, 8, 1e-9)])
def test_layer_norm_window_fp64_matches_oracle(name, N, h, tol):
    W, ad, cd, a_ln, c_ln = _case(name, N)
    print(f"[layer norm] {name} fp64 N={N} h={h}", flush=True)
    _, f, a = _run(W, ad, cd, a_ln, c_ln, N, h, "fp64", ckpt_interval=4)
    ref = oracle_window_grads(W["model"], W["s0"][:N], h, W["actor"], W["critic"], want_theta=True,
                              actor_ln=a_ln, critic_ln=c_ln)
    for key in ("s_h", "obs", "actions", "rewards", "value"):
        assert relnorm(f[key], ref[key]) < tol, key
    assert abs(f["loss"][0] - ref["loss"]) < tol * abs(ref["loss"])
    assert relnorm(a["dL_da"], ref["dL_da"]) < tol
    assert relnorm(a["dL_ds0"], ref["dL_ds0"]) < tol
    assert relnorm(a["dL_dtheta_flat"], _theta_ref(ref)) < tol


def test_layer_norm_changes_the_window_and_fp32_meets_the_bar():
    """Ant, FP32 at the gate's short horizon: the layer-normalised window against the oracle at
    the spec bar, and different from the window without normalisation."""
    W, ad, cd, a_ln, c_ln = _case("ant", 64)
    h = 4
    print("[layer norm] ant fp32 N=64 h=4", flush=True)
    sim, f, a = _run(W, ad, cd, a_ln, c_ln, 64, h, "fp32", ckpt_interval=4)
    envs = [0, 33]
    ref = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], n_total=64,
                              actor_ln=a_ln, critic_ln=c_ln)
    assert float((np.abs(f["s_h"][envs] - ref["s_h"]).max(1) / np.abs(ref["s_h"]).max(1)).max()) < 1e-4
    for got, want in ((a["dL_da"][:, envs], ref["dL_da"]), (a["dL_ds0"][envs], ref["dL_ds0"])):
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3
    plain = P.Sim(W["model"], 64, h, ad, cd, ckpt_interval=4)
    fp = plain.forward(W["s0"], W["actor"], W["critic"])
    torch.cuda.synchronize()
    assert relnorm(fp["actions"].double().cpu().numpy(), f["actions"]) > 1e-2


def test_layer_norm_paths_bitwise_and_critic_values():
    """The tape path, the factor cache and the plain path run the same normalised arithmetic
    as the checkpointed path (bitwise); the critic calls of the learning episode refuse a
    normalised handle."""
    W, ad, cd, a_ln, c_ln = _case("ant", 64)
    h = 3
    print("[layer norm] ant fp32 paths", flush=True)
    sim, f0, a0 = _run(W, ad, cd, a_ln, c_ln, 64, h, "fp32", ckpt_interval=4)
    for kw in (dict(path=P.PATH_TAPE), dict(ckpt_interval=4, factor_cache=True), dict(path=P.PATH_PLAIN)):
        _, f1, a1 = _run(W, ad, cd, a_ln, c_ln, 64, h, "fp32", **kw)
        for key in f0:
            assert np.array_equal(f0[key], f1[key]), (kw, key)
        for key in a0:
            assert np.array_equal(a0[key], a1[key]), (kw, key)
    # the critic calls of the learning episode do not take the normalised networks
    with pytest.raises(P.SimError) as e:
        sim.critic_values(torch.zeros(4, W["obs_dim"], device="cuda"), W["critic"])
    assert "layer normalisation" in str(e.value)
