"""Early termination inside the window (App. A.3 heights; Sec. 3.3 discount restart): the
GPU window against the FP64 oracle, bitwise agreement of the persistent and tape paths,
and no change when no env terminates."""
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


def _case(name, N, low):
    W = wl.workload(name, N)
    md = wl.with_termination(W["model"])
    s0 = W["s0"].copy()
    s0[::2, 2] = low                     # every other env starts below the termination height
    reset = wl.initial_states(md, N, seed=9)
    reset[::4, 2] = low                  # and every fourth restarts below it: a reset each frame
    return W, md, s0, reset


def _run(W, md, s0, reset, h, **kw):
    od = W["obs_dim"]
    N = s0.shape[0]
    sim = P.Sim(md, N, h, [od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]], **kw)
    fw = sim.forward(s0, W["actor"], W["critic"], reset_states=reset)
    ad = sim.adjoint(fw)
    torch.cuda.synchronize()
    f = {k: fw[k].double().cpu().numpy() for k in ("s_h", "actions", "rewards", "value", "done")}
    a = {k: ad[k].double().cpu().numpy() for k in ("dL_da", "dL_ds0")}
    return f, a


@pytest.mark.parametrize("path", ["persistent", "tape"])
def test_termination_fp64_matches_oracle(path):
    W, md, s0, reset = _case("ant", 8, 0.2)
    h = 5
    print(f"[term] ant fp64 {path}", flush=True)
    kw = dict(path=P.PATH_TAPE) if path == "tape" else dict(ckpt_interval=4)
    f, a = _run(W, md, s0, reset, h, precision="fp64", **kw)
    ref = oracle_window_grads(md, s0, h, W["actor"], W["critic"], reset_states=reset)
    assert ref["done"][0].any() and ref["done"][1:].any() and not ref["done"].all()
    assert np.array_equal(f["done"].astype(bool), ref["done"])
    for key in ("s_h", "actions", "rewards"):
        assert relnorm(f[key], ref[key]) < 1e-10, key
    assert relnorm(a["dL_da"], ref["dL_da"]) < 1e-9
    assert relnorm(a["dL_ds0"], ref["dL_ds0"]) < 1e-9


def test_termination_paths_bitwise_and_inactive_is_unchanged():
    W, md, s0, reset = _case("ant", 64, 0.2)
    h = 4
    print("[term] ant fp32 persistent / tape", flush=True)
    f0, a0 = _run(W, md, s0, reset, h, ckpt_interval=4)
    f1, a1 = _run(W, md, s0, reset, h, path=P.PATH_TAPE)
    assert f0["done"].any()
    for key in ("s_h", "actions", "rewards", "done"):
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
