"""The compact per-environment layout with 16, 32 or 64 lanes per environment (several small
envs per wavefront, more wavefronts per CU) against the full layout with one environment per
wavefront, through the C ABI.  The same arithmetic runs in the same order per environment, so
every output and gradient is compared bitwise; the full layout is the one checked against the
FP64 oracle (test_gpu_parity.py)."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads

pytestmark = pytest.mark.gpu

FWD_KEYS = ("s_h", "obs", "actions", "rewards", "value", "loss_env", "loss", "adhesive_count",
            "fp64_refactor_count", "nonfinite")


def _np(d):
    return {k: v.double().cpu().numpy() for k, v in d.items() if torch.is_tensor(v)}


def _run(W, N, h, lanes, **kw):
    od = W["obs_dim"]
    extra = {k: kw.pop(k) for k in ("noise", "log_std", "reset_states", "obs_norm") if k in kw}
    sim = P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                [od] + [w.shape[0] for w, _ in W["critic"]], policy_grad=True, lanes_per_env=lanes, **kw)
    fw = sim.forward(W["s0"][:N], W["actor"], W["critic"], **extra)
    ad = sim.adjoint(fw, want_theta=True)
    torch.cuda.synchronize()
    return _np(fw), _np(ad)


CASES = [("cartpole", 64, 8, dict(ckpt_interval=4)),
         ("cartpole", 64, 4, dict(path=P.PATH_TAPE)),
         ("ant", 64, 3, dict(ckpt_interval=16)),
         ("ant", 64, 3, dict(ckpt_interval=4)),
         ("ant", 64, 2, dict(path=P.PATH_TAPE))]


@pytest.mark.parametrize("name,N,h,kw", CASES, ids=[f"{c[0]}-{'tape' if 'path' in c[3] else 'k' + str(c[3]['ckpt_interval'])}"
                                                   for c in CASES])
def test_compact_layout_bitwise_equals_full_layout(name, N, h, kw):
    W = wl.workload(name, N)
    print(f"[compact] {name} N={N} h={h} {kw} full layout", flush=True)
    f0, a0 = _run(W, N, h, 0, **dict(kw))
    for lanes in (64, 32, 16):
        print(f"[compact] {name} lanes={lanes}", flush=True)
        f1, a1 = _run(W, N, h, lanes, **dict(kw))
        for key in FWD_KEYS:
            assert np.array_equal(f0[key], f1[key]), (lanes, key)
        for key in ("dL_da", "dL_ds0", "dL_dtheta_flat"):
            assert np.array_equal(a0[key], a1[key]), (lanes, key)


def test_compact_layout_with_termination_noise_and_normalisation_bitwise():
    """Early termination (a quarter of the envs restart every frame), the stochastic policy and
    observation normalisation at once, 16 lanes per env against the full layout."""
    W = wl.workload("ant", 64)
    md = wl.with_termination(W["model"])
    W = dict(W, model=md)
    N, h = 64, 4
    s0 = W["s0"].copy()
    s0[::4, 2] = 0.2
    W["s0"] = s0
    rng = np.random.default_rng(6)
    kw = dict(ckpt_interval=4, noise=rng.standard_normal((h, N, 8)), log_std=np.full(8, -0.5),
              reset_states=wl.initial_states(md, N, seed=9),
              obs_norm=(rng.normal(0, 0.1, 37), rng.uniform(0.5, 2.0, 37)))
    print("[compact] ant termination + noise + normalisation", flush=True)
    f0, a0 = _run(W, N, h, 0, **dict(kw))
    f1, a1 = _run(W, N, h, 16, **dict(kw))
    assert f0["done"].any()
    for key in FWD_KEYS + ("done",):
        assert np.array_equal(f0[key], f1[key]), key
    for key in ("dL_da", "dL_ds0", "dL_dtheta_flat", "dL_dlog_std"):
        assert np.array_equal(a0[key], a1[key]), key


def test_compact_layout_fp32_matches_oracle_cartpole():
    """CartPole, 16 lanes per env, the full h = 32 window against the FP64 oracle at the FP32
    bar (states 1e-4, gradient cosine 0.999 and relative norm 1e-3)."""
    W = wl.workload("cartpole", 64)
    h = 32
    print("[compact] cartpole h=32 lanes=16 vs oracle", flush=True)
    f, a = _run(W, 64, h, 16, ckpt_interval=4)
    envs = [0, 17, 42, 63]
    ref = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], n_total=64)
    assert float((np.abs(f["s_h"][envs] - ref["s_h"]).max(1) / np.abs(ref["s_h"]).max(1)).max()) < 1e-4
    for got, want in ((a["dL_da"][:, envs], ref["dL_da"]), (a["dL_ds0"][envs], ref["dL_ds0"])):
        c = float(got.ravel() @ want.ravel() / (np.linalg.norm(got) * np.linalg.norm(want)))
        assert c >= 0.999 and np.linalg.norm(got - want) <= 1e-3 * np.linalg.norm(want)


def test_group_with_compact_members_matches_members():
    """A mixed group: humanoid (full layout), Ant (16 lanes per env) and CartPole (32 lanes),
    one graph-captured launch per direction, bitwise equal to the members' own calls."""
    h = 2
    members = [("humanoid", 24, 0, dict(ckpt_interval=16)), ("ant", 40, 16, dict(path=P.PATH_TAPE)),
               ("cartpole", 48, 32, dict(ckpt_interval=4))]
    sims, args, solo = [], [], []
    for name, N, lanes, kw in members:
        W = wl.workload(name, N)
        od = W["obs_dim"]
        sim = P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                    [od] + [w.shape[0] for w, _ in W["critic"]], lanes_per_env=lanes, **kw)
        a = (sim._dev(W["s0"]), sim.weights(W["actor"]), sim.weights(W["critic"]))
        print(f"[compact group] member {name} lanes={lanes}", flush=True)
        fw = sim.forward(*a)
        solo.append((_np(fw), _np(sim.adjoint(fw))))
        sims.append(sim)
        args.append(a)
    torch.cuda.synchronize()
    G = P.Group(sims)
    print("[compact group] group launch", flush=True)
    gf = G.forward(args)
    ga = G.adjoint(gf)
    torch.cuda.synchronize()
    for i in range(len(members)):
        for key in ("s_h", "actions", "rewards", "value"):
            assert np.array_equal(_np(gf[i])[key], solo[i][0][key]), (i, key)
        for key in ("dL_da", "dL_ds0"):
            assert np.array_equal(_np(ga[i])[key], solo[i][1][key]), (i, key)


def test_autotuner_chooses_among_layouts():
    """For CartPole the tuner times the full layout and the compact one at 64, 32 and 16 lanes
    per env, each on the tape path and every checkpoint interval with and without the factor
    cache, and reports its choice."""
    W = wl.workload("cartpole", 256)
    od = W["obs_dim"]
    print("[compact] tuner cartpole 256", flush=True)
    r = P.tune(W["model"], 256, 4, [od] + [w.shape[0] for w, _ in W["actor"]],
               [od] + [w.shape[0] for w, _ in W["critic"]], W["s0"], W["actor"], W["critic"],
               budget_bytes=1 << 34, reps=1)
    n_k = sum(1 for k in range(1, 5) if 4 % k == 0)                 # S = 4
    assert r["n_candidates"] == 4 * (1 + 2 * n_k)
    assert r["lanes_per_env"] in (0, 16, 32, 64)
