"""Mixed-morphology groups (one graph-captured launch over several models) and the
autotuner, through the C ABI.

The group kernel runs each model's own DOF-specialised window body, so its results are
compared bitwise with the members' own sim_forward_window / sim_adjoint_window calls;
graph replays are compared bitwise with the eager result, with unrelated eager work and
synchronisation between the replays, and after the arguments change (recapture).
"""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl

pytestmark = pytest.mark.gpu

MEMBERS = [("cartpole", 48, None), ("ant", 40, P.PATH_TAPE), ("humanoid", 24, 16)]


def _members(h, precision="fp32", policy_grad=False):
    sims, args = [], []
    for name, n, path in MEMBERS:
        W = wl.workload(name, n)
        od = W["obs_dim"]
        kw = dict(path=path) if path == P.PATH_TAPE else dict(ckpt_interval=path)
        sim = P.Sim(W["model"], n, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                    [od] + [w.shape[0] for w, _ in W["critic"]], precision=precision,
                    policy_grad=policy_grad, **kw)
        sims.append(sim)
        args.append((sim._dev(W["s0"]), sim.weights(W["actor"]), sim.weights(W["critic"])))
    return sims, args


def _np(d):
    return {k: v.double().cpu().numpy() for k, v in d.items() if torch.is_tensor(v)}


def test_group_matches_members_bitwise_and_orders_by_cost():
    h = 3
    sims, args = _members(h, policy_grad=True)
    print("[group] cartpole 48 + ant 40 (tape) + humanoid 24 (k=16), h=3", flush=True)
    solo_f, solo_a = [], []
    for sim, a in zip(sims, args):
        fw = sim.forward(*a)
        ad = sim.adjoint(fw, want_theta=True)
        solo_f.append(fw)
        solo_a.append(ad)
    torch.cuda.synchronize()
    G = P.Group(sims)
    assert G.order() == [2, 1, 0]          # humanoid, ant, cartpole: decreasing per-env cost
    gf = G.forward(args)
    ga = G.adjoint(gf, want_theta=True)
    torch.cuda.synchronize()
    for i in range(len(sims)):
        a, b = _np(solo_f[i]), _np(gf[i])
        for key in ("s_h", "obs", "actions", "rewards", "value", "loss_env", "loss"):
            assert np.array_equal(a[key], b[key]), (i, key)
        a, b = _np(solo_a[i]), _np(ga[i])
        for key in ("dL_da", "dL_ds0", "dL_dtheta_flat"):
            assert np.array_equal(a[key], b[key]), (i, key)


def test_group_graph_replays_and_recapture():
    h = 2
    sims, args = _members(h)
    G = P.Group(sims)
    print("[group graph] eager reference", flush=True)
    ref_f, ref_a = [], []
    for sim, a in zip(sims, args):
        fw = sim.forward(*a)
        ref_f.append(_np(fw))
        ref_a.append(_np(sim.adjoint(fw)))
    torch.cuda.synchronize()
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        print(f"[group graph] replay {rep}", flush=True)
        gf = G.forward(args)
        ga = G.adjoint(gf)
        torch.cuda.synchronize()
        for i in range(len(sims)):
            assert np.array_equal(_np(gf[i])["s_h"], ref_f[i]["s_h"]), (rep, i)
            assert np.array_equal(_np(ga[i])["dL_da"], ref_a[i]["dL_da"]), (rep, i)
            assert np.array_equal(_np(ga[i])["dL_ds0"], ref_a[i]["dL_ds0"]), (rep, i)
        assert G.captures() == 2           # one forward and one adjoint graph, replayed
        y = (x * 2.0).sum()                # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
    # new inputs: the group captures again and follows them
    print("[group graph] recapture on new s0", flush=True)
    args2 = [(a[0] * 1.0001, a[1], a[2]) for a in args]
    gf = G.forward(args2)
    torch.cuda.synchronize()
    assert G.captures() == 3
    for i, (sim, a) in enumerate(zip(sims, args2)):
        solo = sim.forward(*a)
        torch.cuda.synchronize()
        assert np.array_equal(_np(gf[i])["s_h"], _np(solo)["s_h"]), i


def test_group_rejects_mixed_precision_plain_and_duplicates():
    W = wl.workload("cartpole", 8)
    od = W["obs_dim"]
    dims = ([od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]])
    a = P.Sim(W["model"], 8, 2, *dims)
    b = P.Sim(W["model"], 8, 2, *dims, precision="fp64")
    c = P.Sim(W["model"], 8, 2, *dims, path=P.PATH_PLAIN)
    for members, code in (([a, b], -1), ([a, c], -6), ([a, a], -1)):
        with pytest.raises(P.SimError) as e:
            P.Group(members)
        assert e.value.code == code


def test_autotuner_picks_a_valid_configuration():
    W = wl.workload("ant", 64)
    od = W["obs_dim"]
    h = 2
    dims = ([od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]])
    print("[tune] ant 64 h=2, unlimited budget", flush=True)
    r = P.tune(W["model"], 64, h, *dims, W["s0"], W["actor"], W["critic"], budget_bytes=1 << 40, reps=2)
    divisors = [k for k in range(1, 17) if 16 % k == 0]
    # the full layout and the compact one at 64, 32 and 16 lanes per env, each on the tape path
    # and every checkpoint interval with and without the factor cache
    assert r["n_candidates"] == 4 * (2 * len(divisors) + 1)
    assert r["factor_cache"] in (0, 1)
    assert r["path"] in (P.PATH_TAPE, P.PATH_PERSISTENT) and r["ms_window"] > 0
    assert r["lanes_per_env"] in (0, 16, 32, 64)
    # a budget below every tape path's workspace leaves only checkpointed configurations
    tape = P.Sim(W["model"], 64, h, *dims, path=P.PATH_TAPE, lanes_per_env=64)
    k1 = P.Sim(W["model"], 64, h, *dims, ckpt_interval=1)
    assert k1.ws_bytes < tape.ws_bytes
    print("[tune] ant 64 h=2, budget below the tape path", flush=True)
    r2 = P.tune(W["model"], 64, h, *dims, W["s0"], W["actor"], W["critic"],
                budget_bytes=(tape.ws_bytes + k1.ws_bytes) // 2, reps=1)
    assert r2["path"] == P.PATH_PERSISTENT and r2["workspace_bytes"] < tape.ws_bytes
    with pytest.raises(P.SimError) as e:
        P.tune(W["model"], 64, h, *dims, W["s0"], W["actor"], W["critic"], budget_bytes=1, reps=1)
    assert e.value.code == -5


def test_group_with_stochastic_normalised_member_matches_members():
    """A group whose Ant member runs the stochastic policy with observation normalisation and
    the policy-parameter gradient (dL/dlog_std included), beside a plain Humanoid member:
    each member bitwise equal to its own calls."""
    h = 3
    rng = np.random.default_rng(17)
    sims, args = [], []
    for name, n, k in (("ant", 40, 4), ("humanoid", 24, 16)):
        W = wl.workload(name, n)
        od = W["obs_dim"]
        sim = P.Sim(W["model"], n, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                    [od] + [w.shape[0] for w, _ in W["critic"]], ckpt_interval=k, policy_grad=True)
        a = dict(s0=sim._dev(W["s0"]), actor=sim.weights(W["actor"]), critic=sim.weights(W["critic"]))
        if name == "ant":
            na = W["model"]["na"]
            a["noise"] = sim._dev(rng.standard_normal((h, n, na)))
            a["log_std"] = sim._dev(rng.uniform(-1.5, -0.5, na))
            a["obs_norm"] = (sim._dev(rng.normal(0.0, 0.5, od)), sim._dev(rng.uniform(0.3, 2.0, od)))
        sims.append(sim)
        args.append(a)
    print("[group] ant 40 (stochastic, normalised) + humanoid 24, h=3", flush=True)
    solo_f, solo_a = [], []
    for sim, a in zip(sims, args):
        fw = sim.forward(**a)
        ad = sim.adjoint(fw, want_theta=True)
        solo_f.append(_np(fw))
        solo_a.append(_np(ad))
    torch.cuda.synchronize()
    G = P.Group(sims)
    gf = G.forward(args)
    ga = G.adjoint(gf, want_theta=True)
    torch.cuda.synchronize()
    for i in range(2):
        b = _np(gf[i])
        for key in ("s_h", "obs", "actions", "rewards", "value", "loss_env", "loss"):
            assert np.array_equal(solo_f[i][key], b[key]), (i, key)
        b = _np(ga[i])
        keys = ("dL_da", "dL_ds0", "dL_dtheta_flat") + (("dL_dlog_std",) if i == 0 else ())
        for key in keys:
            assert np.array_equal(solo_a[i][key], b[key]), (i, key)
