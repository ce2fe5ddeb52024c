"""Observation normalisation with running statistics (Sec. 3.3): the statistics update, the
window with normalised network inputs (forward, adjoint and policy-parameter gradient) and
the critic calls, through the C-ABI against the FP64 oracle; identity statistics leave every
launch form bitwise unchanged."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads, normalize_obs
from oracle import learn as OL

pytestmark = pytest.mark.gpu


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def _stats(od, seed=4):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.5, od), rng.uniform(0.3, 2.0, od)


def _sim(W, N, h, **kw):
    od = W["obs_dim"]
    return P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                 [od] + [w.shape[0] for w, _ in W["critic"]], **kw)


def _run(sim, W, obs_norm, want_theta=True):
    fw = sim.forward(W["s0"][:sim.N], W["actor"], W["critic"], obs_norm=obs_norm)
    ad = sim.adjoint(fw, want_theta=want_theta)
    torch.cuda.synchronize()
    f = {k: fw[k].double().cpu().numpy() for k in ("s_h", "obs", "actions", "rewards", "value")}
    a = {k: ad[k].double().cpu().numpy() for k in ("dL_da", "dL_ds0")}
    if want_theta:
        a["theta"] = ad["dL_dtheta_flat"].double().cpu().numpy()
    return f, a


@pytest.mark.parametrize("name,N,h,kw", [("ant", 8, 4, dict(ckpt_interval=4)), ("ant", 8, 4, dict(path=P.PATH_TAPE)),
                                         ("humanoid", 2, 2, dict(ckpt_interval=16))],
                         ids=["ant-k4", "ant-tape", "humanoid-k16"])
def test_normalised_window_fp64_matches_oracle(name, N, h, kw):
    W = wl.workload(name, N)
    mu, sc = _stats(W["obs_dim"])
    print(f"[obs-norm] {name} N={N} h={h} {kw}", flush=True)
    sim = _sim(W, N, h, precision="fp64", policy_grad=True, **kw)
    f, a = _run(sim, W, (mu, sc))
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], want_theta=True, obs_norm=(mu, sc))
    want_theta = np.concatenate([x.ravel() for pair in ref["dL_dtheta"] for x in pair])
    for key in ("s_h", "obs", "actions", "rewards", "value"):
        assert relnorm(f[key], ref[key]) < 1e-10, key
    for got, want in ((a["dL_da"], ref["dL_da"]), (a["dL_ds0"], ref["dL_ds0"]), (a["theta"], want_theta)):
        assert relnorm(got, want) < 1e-9
    # and the normalisation changes the window (the statistics are not an identity)
    raw = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"])
    assert relnorm(raw["actions"], ref["actions"]) > 1e-3


def test_identity_statistics_are_bitwise_neutral():
    """mean 0 and inv_std 1 reproduce the raw window bitwise on the persistent, tape and
    plain paths (the normalisation is (o - 0) * 1 = o exactly)."""
    W = wl.workload("humanoid", 64)
    od = W["obs_dim"]
    ident = (np.zeros(od), np.ones(od))
    for kw in (dict(ckpt_interval=4), dict(path=P.PATH_TAPE), dict(path=P.PATH_PLAIN)):
        print(f"[obs-norm] identity humanoid N=64 h=3 {kw}", flush=True)
        sim = _sim(W, 64, 3, policy_grad=True, **kw)
        f0, a0 = _run(sim, W, None)
        f1, a1 = _run(sim, W, ident)
        for key in f0:
            assert np.array_equal(f0[key], f1[key]), (kw, key)
        for key in a0:
            assert np.array_equal(a0[key], a1[key]), (kw, key)
        sim.close()


def test_normalised_paths_bitwise():
    W = wl.workload("ant", 64)
    stats = _stats(W["obs_dim"], seed=6)
    outs = []
    for kw in (dict(ckpt_interval=4), dict(ckpt_interval=1), dict(path=P.PATH_TAPE), dict(path=P.PATH_PLAIN)):
        print(f"[obs-norm] ant N=64 h=4 fp32 {kw}", flush=True)
        sim = _sim(W, 64, 4, policy_grad=True, **kw)
        outs.append(_run(sim, W, stats))
        sim.close()
    for f, a in outs[1:]:
        for key in f:
            assert np.array_equal(f[key], outs[0][0][key]), key
        for key in a:
            assert np.array_equal(a[key], outs[0][1][key]), key


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-12), (torch.float32, 1e-6)])
def test_obs_stats_update_matches_oracle(dt, tol):
    """Three merges of uneven batches (one of them the headline window's 33 x 1024 rows)."""
    rng = np.random.default_rng(12)
    od = 76
    loc, scale = rng.normal(size=od), rng.uniform(0.1, 4.0, od)
    batches = [rng.normal(loc, scale, size=(n, od)) for n in (33 * 1024, 7, 1500)]
    mean = torch.zeros(od, dtype=dt, device="cuda")
    var = torch.zeros(od, dtype=dt, device="cuda")
    inv = torch.zeros(od, dtype=dt, device="cuda")
    count, rc, rm, rv = 0, 0, None, None
    for b in batches:
        x = torch.as_tensor(b, dtype=dt, device="cuda").contiguous()
        count = P.obs_stats_update(x, count, mean, var, inv, eps=1e-5)
        rc, rm, rv, ri = OL.obs_stats_update(x.double().cpu(), rc, rm, rv, 1e-5)
    torch.cuda.synchronize()
    assert count == rc == sum(b.shape[0] for b in batches)
    assert relnorm(mean.double().cpu().numpy(), rm.numpy()) < tol
    assert relnorm(var.double().cpu().numpy(), rv.numpy()) < tol
    assert relnorm(inv.double().cpu().numpy(), ri.numpy()) < tol


@pytest.mark.parametrize("precision,tol,adam_eps,fit_tol",
                         [("fp64", 1e-12, 1e-8, 1e-8), ("fp32", 1e-5, 1e-8, 1e-4), ("fp32", 1e-5, 1e-3, 1e-4)])
def test_normalised_critic_values_and_fit_match_oracle(precision, tol, adam_eps, fit_tol):
    """Critic values and eight Adam steps of the critic fit against the oracle on normalised
    rows.  The FP32 weight change is held to the bar of the FP32 losses (1e-4 relative norm),
    for Adam's usual eps and for a large eps under which the step is a smooth function of the
    gradient (measured: 2e-6 and 3e-6)."""
    W = wl.workload("humanoid", 64)
    h, N = 4, 64
    sim = _sim(W, N, h, ckpt_interval=16, precision=precision)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    torch.cuda.synchronize()
    mu, sc = _stats(sim.od, seed=8)
    print(f"[obs-norm] critic values + fit {precision}", flush=True)
    obs_all = fw["obs"].reshape(-1, sim.od)
    vals = sim.critic_values(obs_all, W["critic"], obs_norm=(mu, sc))
    nobs = normalize_obs(obs_all.double().cpu(), (mu, sc))
    ref_v = OL.critic_values(W["critic"], nobs)
    torch.cuda.synchronize()
    assert relnorm(vals.double().cpu().numpy(), ref_v.numpy()) < tol
    rows = h * N
    obs = fw["obs"][:h].reshape(rows, sim.od)
    tgt = vals.reshape(h + 1, N)[1:].reshape(rows).clone()
    rng = np.random.default_rng(3)
    perm = np.stack([rng.permutation(rows) for _ in range(4)]).astype(np.int32)
    crit = [(torch.as_tensor(Wl, dtype=sim.dtype, device="cuda").contiguous(),
             torch.as_tensor(bl, dtype=sim.dtype, device="cuda").contiguous()) for Wl, bl in W["critic"]]
    n = sum(Wl.size + bl.size for Wl, bl in W["critic"])
    m = torch.zeros(n, dtype=sim.dtype, device="cuda")
    v = torch.zeros(n, dtype=sim.dtype, device="cuda")
    losses = sim.critic_fit(obs, tgt, torch.as_tensor(perm), 2, crit, m, v, 0, 5e-4, eps=adam_eps, obs_norm=(mu, sc))
    torch.cuda.synchronize()
    zeros = [np.zeros_like(x) for Wl, bl in W["critic"] for x in (Wl, bl)]
    ref_layers, _, _, ref_losses = OL.critic_fit(W["critic"], normalize_obs(obs.double().cpu(), (mu, sc)),
                                                 tgt.double().cpu(), perm, 2, zeros, zeros, 0, 5e-4, 0.7, 0.95, adam_eps)
    got_w = np.concatenate([x.double().cpu().numpy().ravel() for pair in crit for x in pair])
    want_w = np.concatenate([x.numpy().ravel() for pair in ref_layers for x in pair])
    init_w = np.concatenate([x.ravel() for pair in W["critic"] for x in pair])
    assert relnorm(losses.double().cpu().numpy(), ref_losses) < (1e-9 if precision == "fp64" else 1e-4)
    err = relnorm(got_w - init_w, want_w - init_w)
    print(f"[obs-norm] critic fit {precision} eps={adam_eps}: weight-change relnorm {err:.3e}", flush=True)
    assert err < fit_tol


def _cos(x, y):
    x, y = np.asarray(x, np.float64).ravel(), np.asarray(y, np.float64).ravel()
    return float(x @ y / (np.linalg.norm(x) * np.linalg.norm(y)))


@pytest.mark.parametrize("name,N,h,k", [("mtu", 2, 2, 16), ("ant", 8, 4, 16)])
def test_normalised_bf16_mlps_match_oracle_bf16_emulation(name, N, h, k):
    """Normalised inputs into the BF16 matrix-core MLPs: the input is normalised in FP32 and
    then rounded to BF16, as the oracle's BF16 emulation normalises and then rounds; the bar
    is that of the unnormalised BF16 test (states 1e-4, gradient cosine 0.999, relative norm
    1e-3)."""
    W = wl.workload(name, N)
    stats = _stats(W["obs_dim"], seed=10)
    print(f"[obs-norm bf16] {name} N={N} h={h}", flush=True)
    sim = _sim(W, N, h, ckpt_interval=k, mlp_precision="bf16")
    f, a = _run(sim, W, stats, want_theta=False)
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=N, bf16=True, obs_norm=stats)
    assert float((np.abs(f["s_h"] - ref["s_h"]).max(1) / np.abs(ref["s_h"]).max(1)).max()) < 1e-4
    assert relnorm(f["actions"], ref["actions"]) < 1e-4
    assert relnorm(f["value"], ref["value"]) < 1e-4
    for got, want in ((a["dL_da"], ref["dL_da"]), (a["dL_ds0"], ref["dL_ds0"])):
        assert _cos(got, want) >= 0.999 and relnorm(got, want) <= 1e-3
