"""The allocation-free critic values (sim_critic_values_noalloc) against sim_critic_values,
through the C ABI: two calls in a row on the same GPU, the second with fewer rows, and a
request beyond the static scratch refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2204_07137_amd as P
import workloads as wl

pytestmark = pytest.mark.gpu


def _ptrs(layers, idx):
    arr = (ctypes.c_void_p * P.MAXL)()
    for i, pair in enumerate(layers):
        arr[i] = pair[idx].data_ptr()
    return arr


def _values_both(sim, obs, critic, obs_norm):
    L = P.lib()
    rows = obs.shape[0]
    ws = sim.critic_workspace(rows)
    w, b = _ptrs(critic, 0), _ptrs(critic, 1)
    pm = ps = None
    if obs_norm is not None:
        pm, ps = (ctypes.c_void_p(x.data_ptr()) for x in obs_norm)
    ref = torch.full((rows,), float("nan"), device="cuda", dtype=sim.dtype)
    got = torch.full((rows,), float("nan"), device="cuda", dtype=sim.dtype)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P._check(L.sim_critic_values(sim.h, ctypes.c_void_p(obs.data_ptr()), rows, w, b, pm, ps,
                                 ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(), st))
    P._check(L.sim_critic_values_noalloc(sim.h, ctypes.c_void_p(obs.data_ptr()), rows, w, b, pm, ps,
                                         ctypes.c_void_p(got.data_ptr()), st))
    torch.cuda.synchronize()
    return got.double().cpu().numpy(), ref.double().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_critic_values_noalloc_matches_workspace_call(precision):
    W = wl.workload("humanoid", 256)
    od = W["obs_dim"]
    h = 8
    sim = P.Sim(W["model"], 256, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                [od] + [w.shape[0] for w, _ in W["critic"]], ckpt_interval=16, precision=precision)
    fw = sim.forward(W["s0"], W["actor"], W["critic"])
    torch.cuda.synchronize()
    critic = sim.weights(W["critic"])
    rng = np.random.default_rng(5)
    norm = (sim._dev(rng.normal(size=od)), sim._dev(rng.uniform(0.5, 2.0, size=od)))
    obs_all = fw["obs"].reshape(-1, od).contiguous()             # (h + 1) N = 2304 rows
    for rows, obs_norm in ((obs_all.shape[0], norm), (37, None)):
        print(f"[noalloc] {precision} rows={rows} normalised={obs_norm is not None}", flush=True)
        got, ref = _values_both(sim, obs_all[:rows].contiguous(), critic, obs_norm)
        assert np.isfinite(ref).all()
        assert np.array_equal(got, ref)                           # same kernels, same order


def test_critic_values_noalloc_rejects_rows_beyond_the_scratch():
    W = wl.workload("humanoid", 4)
    od = W["obs_dim"]
    sim = P.Sim(W["model"], 4, 2, None, [od] + [w.shape[0] for w, _ in W["critic"]], ckpt_interval=16)
    critic = sim.weights(W["critic"])
    rows = 70000                          # hidden activations 70000 x (128 + 128) x 4 B > 64 MiB
    obs = torch.zeros(rows, od, device="cuda")           # inputs and outputs sized for the rows
    out = torch.zeros(rows, device="cuda")
    L = P.lib()
    rc = L.sim_critic_values_noalloc(sim.h, ctypes.c_void_p(obs.data_ptr()), rows, _ptrs(critic, 0),
                                     _ptrs(critic, 1), None, None, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -5 and "static scratch" in L.sim_last_error().decode()
    torch.cuda.synchronize()
