"""GPU learning-episode update (Adam, target critic, TD-lambda, critic values and fit)
through the C-ABI against the FP64 oracle of oracle/learn.py."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import learn as OL

pytestmark = pytest.mark.gpu


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def _cuda(x, dt):
    return torch.as_tensor(np.asarray(x), dtype=dt, device="cuda").contiguous()


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
def test_adam_and_soft_update_match_oracle(dt, tol):
    rng = np.random.default_rng(1)
    shapes = [(64, 37), (64,), (8, 64), (8,)]
    ps = [rng.normal(size=s) for s in shapes]
    gs = [rng.normal(size=s) for s in shapes]
    ms = [rng.normal(size=s) * 0.1 for s in shapes]
    vs = [np.abs(rng.normal(size=s)) * 0.1 for s in shapes]
    params = [_cuda(p, dt) for p in ps]
    flat = lambda xs: _cuda(np.concatenate([x.ravel() for x in xs]), dt)
    g, m, v = flat(gs), flat(ms), flat(vs)
    P.adam_step(params, g, m, v, step=5, lr=0.002, beta1=0.7, beta2=0.95, eps=1e-8)
    Pr, Mr, Vr = OL.adam_step(ps, gs, ms, vs, 5, 0.002, 0.7, 0.95, 1e-8)
    torch.cuda.synchronize()
    for a, b in zip(params, Pr):
        assert relnorm(a.double().cpu().numpy(), b.numpy()) < tol
    assert relnorm(m.double().cpu().numpy(), np.concatenate([x.numpy().ravel() for x in Mr])) < tol
    assert relnorm(v.double().cpu().numpy(), np.concatenate([x.numpy().ravel() for x in Vr])) < tol
    tgt = [_cuda(rng.normal(size=s), dt) for s in shapes]
    ref = OL.soft_update([t.double().cpu() for t in tgt], ps, 0.995)
    P.soft_update(tgt, [_cuda(p, dt) for p in ps], 0.995)
    torch.cuda.synchronize()
    for a, b in zip(tgt, ref):
        assert relnorm(a.double().cpu().numpy(), b.numpy()) < tol


def _window(N=64, h=8, precision="fp64"):
    W = wl.workload("humanoid", N)
    od = W["obs_dim"]
    sim = P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                [od] + [w.shape[0] for w, _ in W["critic"]], ckpt_interval=16, precision=precision)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    torch.cuda.synchronize()
    return W, sim, fw


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_critic_values_and_td_lambda_match_oracle(precision, tol):
    W, sim, fw = _window(precision=precision)
    h, N = fw["rewards"].shape
    print(f"[learn] values + td-lambda {precision}", flush=True)
    vals = sim.critic_values(fw["obs"], W["critic"]).reshape(h + 1, N)
    ref_v = OL.critic_values(W["critic"], fw["obs"].double().cpu().reshape(-1, sim.od)).reshape(h + 1, N)
    assert relnorm(vals.double().cpu().numpy(), ref_v.numpy()) < tol
    est = P.td_lambda(fw["rewards"], vals, 0.99, 0.95)
    ref = OL.td_lambda(fw["rewards"].double().cpu(), vals.double().cpu(), 0.99, 0.95)
    torch.cuda.synchronize()
    assert relnorm(est.double().cpu().numpy(), ref.numpy()) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_critic_fit_matches_oracle(precision):
    """16 passes x 4 minibatches (App. A.2) of the humanoid critic on a window's states."""
    W, sim, fw = _window(precision=precision)
    h, N = fw["rewards"].shape
    rows = h * N
    print(f"[learn] critic fit {precision} rows={rows}", flush=True)
    obs = fw["obs"][:h].reshape(rows, sim.od)
    vals = sim.critic_values(fw["obs"], W["critic"]).reshape(h + 1, N)
    tgt = P.td_lambda(fw["rewards"], vals, 0.99, 0.95).reshape(rows)
    rng = np.random.default_rng(2)
    perm = np.stack([rng.permutation(rows) for _ in range(16)]).astype(np.int32)
    crit = [(_cuda(Wl, sim.dtype), _cuda(bl, sim.dtype)) for Wl, bl in W["critic"]]
    n = sum(Wl.size + bl.size for Wl, bl in W["critic"])
    m = torch.zeros(n, dtype=sim.dtype, device="cuda")
    v = torch.zeros(n, dtype=sim.dtype, device="cuda")
    losses = sim.critic_fit(obs, tgt, torch.as_tensor(perm), 4, crit, m, v, 0, 5e-4)
    torch.cuda.synchronize()
    zeros = [np.zeros_like(x) for Wl, bl in W["critic"] for x in (Wl, bl)]
    ref_layers, ref_m, _, ref_losses = OL.critic_fit(W["critic"], obs.double().cpu(), tgt.double().cpu(), perm, 4,
                                                     zeros, zeros, 0, 5e-4, 0.7, 0.95, 1e-8)
    got_w = np.concatenate([x.double().cpu().numpy().ravel() for pair in crit for x in pair])
    want_w = np.concatenate([x.numpy().ravel() for pair in ref_layers for x in pair])
    init_w = np.concatenate([x.ravel() for pair in W["critic"] for x in pair])
    assert relnorm(losses.double().cpu().numpy(), ref_losses) < (1e-9 if precision == "fp64" else 1e-4)
    # compare the change of the weights (64 Adam steps of lr 5e-4)
    tol = 1e-8 if precision == "fp64" else 2e-2
    assert relnorm(got_w - init_w, want_w - init_w) < tol
    assert relnorm(m.double().cpu().numpy(), np.concatenate([x.numpy().ravel() for x in ref_m])) < tol
    # bitwise reproducible
    crit2 = [(_cuda(Wl, sim.dtype), _cuda(bl, sim.dtype)) for Wl, bl in W["critic"]]
    m2, v2 = torch.zeros_like(m), torch.zeros_like(v)
    sim.critic_fit(obs, tgt, torch.as_tensor(perm), 4, crit2, m2, v2, 0, 5e-4)
    torch.cuda.synchronize()
    for (a, b), (c, d) in zip(crit, crit2):
        assert torch.equal(a, c) and torch.equal(b, d)
