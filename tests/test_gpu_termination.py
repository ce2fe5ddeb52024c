"""Early termination inside the window (App. A.3 heights; Sec. 3.3 discount restart): the
GPU window against the FP64 oracle, bitwise agreement of the persistent and tape paths,
and no change when no env terminates."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads
from oracle import learn as OL

pytestmark = pytest.mark.gpu


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def _case(name, N, low):
    W = wl.workload(name, N)
    md = wl.with_termination(W["model"])
    s0 = W["s0"].copy()
    s0[::2, 2] = low                     # every other env starts below the termination height
    reset = wl.initial_states(md, N, seed=9)
    reset[::4, 2] = low                  # and every fourth restarts below it: a reset each frame
    return W, md, s0, reset


def _run(W, md, s0, reset, h, want_theta=False, **kw):
    od = W["obs_dim"]
    N = s0.shape[0]
    sim = P.Sim(md, N, h, [od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]],
                policy_grad=want_theta, **kw)
    fw = sim.forward(s0, W["actor"], W["critic"], reset_states=reset)
    ad = sim.adjoint(fw, want_theta=want_theta)
    torch.cuda.synchronize()
    f = {k: fw[k].double().cpu().numpy() for k in ("s_h", "actions", "rewards", "value", "done", "loss", "loss_env")}
    a = {k: ad[k].double().cpu().numpy() for k in ("dL_da", "dL_ds0")}
    if want_theta:
        a["theta"] = ad["dL_dtheta_flat"].double().cpu().numpy()
    f["_sim"], f["_fw"] = sim, fw
    return f, a


@pytest.mark.parametrize("path", ["persistent", "tape"])
def test_termination_fp64_matches_oracle(path):
    W, md, s0, reset = _case("ant", 8, 0.2)
    h = 5
    print(f"[term] ant fp64 {path}", flush=True)
    kw = dict(path=P.PATH_TAPE) if path == "tape" else dict(ckpt_interval=4)
    f, a = _run(W, md, s0, reset, h, want_theta=True, precision="fp64", **kw)
    ref = oracle_window_grads(md, s0, h, W["actor"], W["critic"], reset_states=reset, want_theta=True)
    assert ref["done"][0].any() and ref["done"][1:].any() and not ref["done"].all()
    assert np.array_equal(f["done"].astype(bool), ref["done"])
    for key in ("s_h", "actions", "rewards", "value"):
        assert relnorm(f[key], ref[key]) < 1e-10, key
    # the window's loss output, with the segment discounts and no value after a last-frame reset
    assert abs(f["loss"][0] - ref["loss"]) < 1e-10 * abs(ref["loss"])
    assert abs(f["loss_env"].sum() - f["loss"][0]) < 1e-12 * abs(ref["loss"])
    want_theta = np.concatenate([x.ravel() for pair in ref["dL_dtheta"] for x in pair])
    for got, want in ((a["dL_da"], ref["dL_da"]), (a["dL_ds0"], ref["dL_ds0"]), (a["theta"], want_theta)):
        assert relnorm(got, want) < 1e-9
    # the critic's TD-lambda targets stop at each termination
    sim, fw = f["_sim"], f["_fw"]
    vals = sim.critic_values(fw["obs"], W["critic"]).reshape(h + 1, 8)
    est = P.td_lambda(fw["rewards"], vals, 0.99, 0.95, done=fw["done"])
    plain = P.td_lambda(fw["rewards"], vals, 0.99, 0.95)
    torch.cuda.synchronize()
    want = OL.td_lambda(fw["rewards"].double().cpu(), vals.double().cpu(), 0.99, 0.95, done=ref["done"]).numpy()
    assert relnorm(est.double().cpu().numpy(), want) < 1e-12
    assert not np.allclose(plain.double().cpu().numpy(), want)


def test_termination_paths_bitwise_and_inactive_is_unchanged():
    W, md, s0, reset = _case("ant", 64, 0.2)
    h = 4
    print("[term] ant fp32 persistent / tape", flush=True)
    f0, a0 = _run(W, md, s0, reset, h, ckpt_interval=4)
    f1, a1 = _run(W, md, s0, reset, h, path=P.PATH_TAPE)
    assert f0["done"].any()
    for key in ("s_h", "actions", "rewards", "value", "done", "loss", "loss_env"):
        assert np.array_equal(f0[key], f1[key]), key
    assert np.array_equal(a0["dL_da"], a1["dL_da"]) and np.array_equal(a0["dL_ds0"], a1["dL_ds0"])
    # standing humanoids do not fall within three frames: termination on or off is the same window
    W = wl.workload("humanoid", 32)
    md = wl.with_termination(W["model"])
    reset = wl.initial_states(md, 32, seed=9)
    print("[term] humanoid inactive", flush=True)
    f2, a2 = _run(W, md, W["s0"], reset, 3, ckpt_interval=4)
    od = W["obs_dim"]
    sim = P.Sim(W["model"], 32, 3, [od] + [w.shape[0] for w, _ in W["actor"]],
                [od] + [w.shape[0] for w, _ in W["critic"]], ckpt_interval=4)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    assert not f2["done"].any()
    assert np.array_equal(f2["s_h"], fw["s_h"].double().cpu().numpy())
    assert np.array_equal(a2["dL_da"], ad["dL_da"].double().cpu().numpy())
    assert np.array_equal(a2["dL_ds0"], ad["dL_ds0"].double().cpu().numpy())


def test_group_with_a_terminating_member_matches_members():
    """A group of an Ant with early termination (tape path) and a Humanoid without it
    (k 16): each member bitwise equal to its own calls, the Ant's done flags included."""
    h = 3
    sims, args = [], []
    for name, n, kw in (("ant", 40, dict(path=P.PATH_TAPE)), ("humanoid", 24, dict(ckpt_interval=16))):
        W = wl.workload(name, n)
        md = W["model"]
        od = W["obs_dim"]
        s0 = W["s0"].copy()
        a = {}
        if name == "ant":
            md = wl.with_termination(md)
            s0[::2, 2] = 0.2
            reset = wl.initial_states(md, n, seed=9)
            reset[::4, 2] = 0.2
        sim = P.Sim(md, n, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                    [od] + [w.shape[0] for w, _ in W["critic"]], **kw)
        a = dict(s0=sim._dev(s0), actor=sim.weights(W["actor"]), critic=sim.weights(W["critic"]))
        if name == "ant":
            a["reset_states"] = sim._dev(reset)
        sims.append(sim)
        args.append(a)
    print("[term group] ant 40 (termination, tape) + humanoid 24 (k=16), h=3", flush=True)
    solo_f, solo_a = [], []
    for sim, a in zip(sims, args):
        fw = sim.forward(**a)
        solo_f.append({k: v.double().cpu().numpy() for k, v in fw.items() if torch.is_tensor(v)})
        ad = sim.adjoint(fw)
        solo_a.append({k: v.double().cpu().numpy() for k, v in ad.items() if torch.is_tensor(v)})
    G = P.Group(sims)
    gf = G.forward(args)
    ga = G.adjoint(gf)
    torch.cuda.synchronize()
    assert solo_f[0]["done"].any() and "done" not in solo_f[1]
    for i in range(2):
        b = {k: v.double().cpu().numpy() for k, v in gf[i].items() if torch.is_tensor(v)}
        for key in ("s_h", "obs", "actions", "rewards", "value") + (("done",) if i == 0 else ()):
            assert np.array_equal(solo_f[i][key], b[key]), (i, key)
        b = {k: v.double().cpu().numpy() for k, v in ga[i].items() if torch.is_tensor(v)}
        for key in ("dL_da", "dL_ds0"):
            assert np.array_equal(solo_a[i][key], b[key]), (i, key)


def test_autograd_window_with_termination_noise_and_normalisation():
    """torch.autograd.Function over an FP64 Ant window that combines early termination, the
    stochastic policy and observation normalisation: the loss (with the segment discounts)
    and the gradients to s0, the actor parameters and log_std match the oracle."""
    N, h = 8, 5
    W, md, s0, reset = _case("ant", N, 0.2)
    od, na = W["obs_dim"], W["model"]["na"]
    rng = np.random.default_rng(21)
    noise = rng.standard_normal((h, N, na))
    log_std = rng.uniform(-1.5, -0.5, na)
    mu, sc = rng.normal(0.0, 0.5, od), rng.uniform(0.3, 2.0, od)
    sim = P.Sim(md, N, h, [od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]],
                ckpt_interval=4, precision="fp64", policy_grad=True)
    dev = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64, device="cuda")
    Fn = P.window_function(noise=dev(noise), reset_states=dev(reset), obs_norm=(dev(mu), dev(sc)))
    s0_t = dev(s0).requires_grad_(True)
    params = [dev(x).requires_grad_(True) for pair in W["actor"] for x in pair] + [dev(log_std).requires_grad_(True)]
    print("[term autograd] ant fp64 termination + noise + obs_norm", flush=True)
    loss, *_ = Fn.apply(sim, s0_t, None, W["critic"], *params)
    loss.backward()
    torch.cuda.synchronize()
    ref = oracle_window_grads(md, s0, h, W["actor"], W["critic"], want_theta=True, noise=noise, log_std=log_std,
                              reset_states=reset, obs_norm=(mu, sc))
    assert ref["done"].any()
    assert abs(float(loss.detach()) - ref["loss"]) < 1e-10 * abs(ref["loss"])
    assert relnorm(s0_t.grad.cpu().numpy(), ref["dL_ds0"]) < 1e-9
    got = np.concatenate([p.grad.cpu().numpy().ravel() for p in params])
    want = np.concatenate([x.ravel() for pair in ref["dL_dtheta"] for x in pair] + [ref["dL_dlog_std"]])
    assert relnorm(got, want) < 1e-9
