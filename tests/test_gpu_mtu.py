"""GPU parity of the muscle-driven models (Hill-type muscle-tendon units) against the
FP64 oracle, through the C ABI.

* The muscle arm (one muscle across a cart-pole hinge, no gravity, open-loop
  excitations, linear critic on the state) over a full 32-frame window: FP64 to
  rounding, FP32 to the state / gradient bar.
* The 152-unit humanoid on short windows (the oracle is slow: ~2 s per env-frame) in
  FP64 and FP32, and at full size (2048 envs, h = 32, FP64) on the first frames of a
  sampled env, which the oracle computes on its own.
* Checkpoint intervals and the tape path bitwise equal; a mixed group with a muscle
  model bitwise equal to the members' own calls.
"""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window, oracle_window_grads

pytestmark = pytest.mark.gpu


def relnorm(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def cosine(x, y):
    x, y = np.asarray(x, np.float64).ravel(), np.asarray(y, np.float64).ravel()
    return float(x @ y / (np.linalg.norm(x) * np.linalg.norm(y)))


def _np(d):
    return {k: v.double().cpu().numpy() for k, v in d.items() if torch.is_tensor(v)}


def _arm(h, precision):
    md = wl.muscle_arm()
    rng = np.random.default_rng(3)
    N = 8
    s0 = np.column_stack([rng.normal(0, 0.1, N), rng.uniform(-0.8, 0.8, N), rng.normal(0, 0.3, N),
                          rng.normal(0, 0.5, N), rng.uniform(0.0, 1.0, N)])
    u = rng.uniform(0.05, 0.95, (h, N, 1))
    critic = [(rng.normal(size=(1, 5)), np.zeros(1))]
    sim = P.Sim(md, N, h, None, [5, 1], ckpt_interval=2, precision=precision)
    fw = sim.forward(s0, None, critic, actions_in=u)
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    ref = oracle_window_grads(md, s0, h, None, critic, actions=u, n_total=N)
    return _np(fw), _np(ad), ref


def test_muscle_arm_fp64_full_window():
    print("[mtu] muscle arm fp64 h=32", flush=True)
    fw, ad, ref = _arm(32, "fp64")
    assert relnorm(fw["s_h"], ref["s_h"]) < 1e-12
    assert relnorm(ad["dL_da"], ref["dL_da"]) < 1e-10
    assert relnorm(ad["dL_ds0"], ref["dL_ds0"]) < 1e-10


def test_muscle_arm_fp32_full_window():
    print("[mtu] muscle arm fp32 h=32", flush=True)
    fw, ad, ref = _arm(32, "fp32")
    assert relnorm(fw["s_h"], ref["s_h"]) < 1e-4
    for got, want in ((ad["dL_da"], ref["dL_da"]), (ad["dL_ds0"], ref["dL_ds0"])):
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3


def _mtu_sim(W, N, h, **kw):
    od = W["obs_dim"]
    return P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                 [od] + [w.shape[0] for w, _ in W["critic"]], **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mtu_humanoid_short_window_matches_oracle(precision):
    W = wl.workload("mtu", 2)
    h = 2
    print(f"[mtu] humanoid 152 muscles, N=2 h=2 {precision}", flush=True)
    sim = _mtu_sim(W, 2, h, ckpt_interval=16, precision=precision)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    fw, ad = _np(fw), _np(ad)
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=2)
    if precision == "fp64":
        for key in ("s_h", "obs", "actions", "rewards", "value"):
            assert relnorm(fw[key], ref[key]) < 1e-10, key
        assert relnorm(ad["dL_da"], ref["dL_da"]) < 1e-8
        assert relnorm(ad["dL_ds0"], ref["dL_ds0"]) < 1e-8
    else:
        sh, rs = fw["s_h"], ref["s_h"]
        assert float((np.abs(sh - rs).max(1) / np.abs(rs).max(1)).max()) < 1e-4
        for got, want in ((ad["dL_da"], ref["dL_da"]), (ad["dL_ds0"], ref["dL_ds0"])):
            assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3


def test_mtu_paths_bitwise_identical():
    W = wl.workload("mtu", 8)
    h = 2
    print("[mtu] paths k=16 / k=1 / tape", flush=True)
    outs = []
    for kw in (dict(ckpt_interval=16), dict(ckpt_interval=1), dict(path=P.PATH_TAPE)):
        sim = _mtu_sim(W, 8, h, **kw)
        fw = sim.forward(W["s0"], W["actor"], W["critic"])
        ad = sim.adjoint(fw)
        torch.cuda.synchronize()
        outs.append((_np(fw), _np(ad)))
    for fw, ad in outs[1:]:
        for key in ("s_h", "obs", "actions", "rewards", "value"):
            assert np.array_equal(fw[key], outs[0][0][key]), key
        assert np.array_equal(ad["dL_da"], outs[0][1]["dL_da"])
        assert np.array_equal(ad["dL_ds0"], outs[0][1]["dL_ds0"])


def test_mtu_full_size_sampled_frames_fp64():
    """2048 envs, h = 32, FP64: the first two frames of env 1234 (observations, actions,
    rewards) against the oracle run on that env alone; the whole batch stays finite."""
    W = wl.workload("mtu")
    N = W["n_envs"]
    print(f"[mtu] full size N={N} h=32 fp64", flush=True)
    sim = _mtu_sim(W, N, W["h"], ckpt_interval=16, precision="fp64")
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    fw, ad = _np(fw), _np(ad)
    assert np.isfinite(ad["dL_da"]).all() and np.isfinite(ad["dL_ds0"]).all()
    assert not fw["nonfinite"].any()
    e = 1234
    ref = oracle_window(W["model"], W["s0"][[e]], 2, W["actor"], W["critic"], n_total=N)
    for t in range(2):
        assert relnorm(fw["actions"][t, e], ref["actions"][t][0].numpy()) < 1e-11
        assert relnorm(fw["rewards"][t, e], ref["rewards"][t].numpy()) < 1e-11
    assert relnorm(fw["obs"][2, e], ref["obs"][2][0].numpy()) < 1e-10


def test_group_with_muscle_model_bitwise():
    h = 2
    members = []
    for name, n in (("mtu", 6), ("ant", 10), ("cartpole", 12)):
        W = wl.workload(name, n)
        sim = _mtu_sim(W, n, h, ckpt_interval=(16 if name != "cartpole" else 4))
        members.append((sim, (sim._dev(W["s0"]), sim.weights(W["actor"]), sim.weights(W["critic"]))))
    print("[mtu] group mtu 6 + ant 10 + cartpole 12", flush=True)
    solo = []
    for sim, a in members:
        fw = sim.forward(*a)
        solo.append((_np(fw), _np(sim.adjoint(fw))))
    torch.cuda.synchronize()
    G = P.Group([s for s, _ in members])
    gf = G.forward([a for _, a in members])
    ga = G.adjoint(gf)
    torch.cuda.synchronize()
    for i in range(3):
        assert np.array_equal(_np(gf[i])["s_h"], solo[i][0]["s_h"]), i
        assert np.array_equal(_np(ga[i])["dL_da"], solo[i][1]["dL_da"]), i
        assert np.array_equal(_np(ga[i])["dL_ds0"], solo[i][1]["dL_ds0"]), i


@pytest.mark.parametrize("name,N,h,k", [("mtu", 2, 2, 16), ("ant", 8, 4, 16)])
def test_bf16_mlp_matches_oracle_bf16_emulation(name, N, h, k):
    """BF16 matrix-core actor and critic (FP32 dynamics) against the oracle's BF16
    emulation (BF16 weights, layer inputs and output adjoints; exact accumulation).  The
    two differ by FP32 accumulation and by the BF16 rounding of hidden values that sit on
    a rounding boundary, so the bar is the FP32 one: states 1e-4, gradient cosine 0.999
    and relative norm 1e-3."""
    W = wl.workload(name, N)
    print(f"[bf16 mlp] {name} N={N} h={h}", flush=True)
    sim = _mtu_sim(W, N, h, ckpt_interval=k, mlp_precision="bf16")
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    fw, ad = _np(fw), _np(ad)
    ref = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=N, bf16=True)
    sh, rs = fw["s_h"], ref["s_h"]
    assert float((np.abs(sh - rs).max(1) / np.abs(rs).max(1)).max()) < 1e-4
    assert relnorm(fw["actions"], ref["actions"]) < 1e-4
    assert relnorm(fw["value"], ref["value"]) < 1e-4
    for got, want in ((ad["dL_da"], ref["dL_da"]), (ad["dL_ds0"], ref["dL_ds0"])):
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3
    # the BF16 policy differs from the FP32 one by far more than the parity above
    ref32 = oracle_window_grads(W["model"], W["s0"], h, W["actor"], W["critic"], n_total=N)
    assert relnorm(fw["actions"], ref32["actions"]) > 10 * relnorm(fw["actions"], ref["actions"])


def test_bf16_muscle_humanoid_full_batch_matches_oracle_bf16_emulation():
    """The configuration's own launch (152-unit humanoid, 2048 envs, k = 16, BF16 networks,
    FP32 dynamics) against the oracle's BF16 emulation on the 4 envs drawn with seed 4, over
    the longest window on which twice the oracle's FP32 storage floor stays under the bar for
    those envs (tests/golden/fp32_floor.json, h_gate): states 1e-4, gradient cosine 0.999 and
    relative norm 1e-3 over the sampled envs together."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "fp32_floor.json")) as fh:
        fl = json.load(fh)["mtu"]
    envs, h, N = fl["envs"], fl["h_gate"], fl["n_envs"]
    W = wl.workload("mtu", N)
    print(f"[bf16 mlp] mtu N={N} h={h} k=16 envs={envs}", flush=True)
    sim = _mtu_sim(W, N, h, ckpt_interval=16, mlp_precision="bf16")
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    fw, ad = _np(fw), _np(ad)
    ref = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], n_total=N, bf16=True)
    sh, rs = fw["s_h"][envs], ref["s_h"]
    assert float((np.abs(sh - rs).max(1) / np.abs(rs).max(1)).max()) < 1e-4
    assert relnorm(fw["actions"][:, envs], ref["actions"]) < 1e-4
    for got, want in ((ad["dL_da"][:, envs], ref["dL_da"]), (ad["dL_ds0"][envs], ref["dL_ds0"])):
        assert cosine(got, want) >= 0.999 and relnorm(got, want) <= 1e-3
