"""Layer normalisation of the hidden layers of the actor and the critic (App. A.2: ELU hidden
layers, each followed by a layer normalisation with a gain and a bias), switched on with
SimOptions.layer_norm: the in-kernel MLPs of the window, their input adjoints, the
policy-parameter gradient (which then includes the gains and biases), and the critic values
and critic fit of the learning episode, against the oracle's layer-normalised MLP
(oracle.window.mlp_forward with ln) and its critic fit (oracle.learn.critic_fit with ln)."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import learn as OL
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


def test_layer_norm_paths_bitwise():
    """The tape path, the factor cache and the plain path run the same normalised arithmetic
    as the checkpointed path (bitwise)."""
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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_layer_norm_critic_values_and_fit_match_oracle(precision):
    """The learning episode's critic calls with normalised hidden layers: the critic's values
    (sim_critic_values_ln) and 4 passes x 4 minibatches of the critic fit, whose Adam moments
    and updates include the gains and biases (library order W, b, g, beta per hidden layer),
    against the oracle's fit of the same normalised critic; the un-normalised entry points
    refuse the handle."""
    W, ad, cd, a_ln, c_ln = _case("ant", 32)
    sim = P.Sim(W["model"], 32, 4, ad, cd, precision=precision, layer_norm=True, ckpt_interval=4)
    rng = np.random.default_rng(5)
    rows = 96
    obs = rng.normal(size=(rows, W["obs_dim"]))
    print(f"[layer norm] critic values and fit, {precision}", flush=True)
    vals = sim.critic_values(obs, W["critic"], critic_ln=c_ln)
    torch.cuda.synchronize()
    ref = OL.critic_values(W["critic"], obs, ln=c_ln).numpy()
    assert relnorm(vals.double().cpu().numpy(), ref) < (1e-12 if precision == "fp64" else 1e-5)
    tgt = rng.normal(size=rows)
    perm = np.stack([rng.permutation(rows) for _ in range(4)]).astype(np.int32)
    crit = [(sim._dev(Wl), sim._dev(bl)) for Wl, bl in W["critic"]]
    cln = [(sim._dev(g), sim._dev(b)) for g, b in c_ln]
    flat0 = []
    for i, (Wl, bl) in enumerate(W["critic"]):
        flat0 += [Wl.ravel(), bl.ravel()]
        if i < len(W["critic"]) - 1:
            flat0 += [c_ln[i][0].ravel(), c_ln[i][1].ravel()]
    n = sum(x.size for x in flat0)
    m = torch.zeros(n, dtype=sim.dtype, device="cuda")
    v = torch.zeros(n, dtype=sim.dtype, device="cuda")
    losses = sim.critic_fit(obs, tgt, torch.as_tensor(perm), 4, crit, m, v, 0, 5e-3, critic_ln=cln)
    torch.cuda.synchronize()
    zeros = []
    for i, (Wl, bl) in enumerate(W["critic"]):
        zeros += [np.zeros_like(Wl), np.zeros_like(bl)]
        if i < len(W["critic"]) - 1:
            zeros += [np.zeros_like(c_ln[i][0]), np.zeros_like(c_ln[i][1])]
    rl, rln, rm, _, rlosses = OL.critic_fit(W["critic"], obs, tgt, perm, 4, zeros, zeros, 0, 5e-3, 0.7, 0.95, 1e-8,
                                            ln=c_ln)
    got, want = [], []
    for i, ((Wg, bg), (Wr, br)) in enumerate(zip(crit, rl)):
        got += [Wg, bg]
        want += [Wr, br]
        if i < len(rl) - 1:
            got += list(cln[i])
            want += list(rln[i])
    got = np.concatenate([x.double().cpu().numpy().ravel() for x in got])
    want = np.concatenate([x.numpy().ravel() for x in want])
    init = np.concatenate(flat0)
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert relnorm(losses.double().cpu().numpy(), rlosses) < tol
    assert relnorm(got - init, want - init) < (1e-8 if precision == "fp64" else 1e-3)
    assert relnorm(m.double().cpu().numpy(), np.concatenate([x.numpy().ravel() for x in rm])) < (
        1e-8 if precision == "fp64" else 1e-3)
    # the entry points without the gains and biases refuse a normalised handle
    with pytest.raises(P.SimError) as e:
        sim.critic_values(obs, W["critic"])
    assert "sim_critic_values_ln" in str(e.value)
