"""Contact diagnostics of the forward window (Sec. 3.1 penalty contact taken literally):
the per-env count of contact evaluations whose normal force pulls, against the FP64
oracle's count, and equal across the launch forms."""
import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl
from oracle import oracle_window_grads

pytestmark = pytest.mark.gpu


def _case(N):
    W = wl.workload("ant", N)
    md = W["model"]
    s0 = W["s0"].copy()
    s0[:, 2] -= 0.05                                    # the foot spheres start 5 cm deep
    s0[:, md["nq"] + 2] = np.linspace(0.0, 7.0, N)       # root rising at 0 .. 7 m/s
    return W, s0


def _sim(W, N, h, **kw):
    od = W["obs_dim"]
    return P.Sim(W["model"], N, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                 [od] + [w.shape[0] for w, _ in W["critic"]], **kw)


def test_adhesive_count_matches_oracle():
    N, h = 8, 2
    W, s0 = _case(N)
    print("[contacts] ant fp64 adhesive count", flush=True)
    sim = _sim(W, N, h, precision="fp64", ckpt_interval=4)
    fw = sim.forward(s0, W["actor"], W["critic"])
    torch.cuda.synchronize()
    got = fw["adhesive_count"].cpu().numpy()
    ref = oracle_window_grads(W["model"], s0, h, W["actor"], W["critic"])
    assert ref["adhesive"].sum() > 0 and (ref["adhesive"] == 0).any()
    assert np.array_equal(got, ref["adhesive"].astype(got.dtype))


def test_adhesive_count_equal_across_launch_forms():
    N, h = 64, 2
    W, s0 = _case(N)
    counts = []
    for kw in (dict(ckpt_interval=4), dict(path=P.PATH_TAPE), dict(path=P.PATH_PLAIN)):
        print(f"[contacts] ant fp32 {kw}", flush=True)
        sim = _sim(W, N, h, **kw)
        fw = sim.forward(s0, W["actor"], W["critic"])
        torch.cuda.synchronize()
        counts.append(fw["adhesive_count"].cpu().numpy())
        sim.close()
    assert counts[0].sum() > 0
    for c in counts[1:]:
        assert np.array_equal(c, counts[0])
