"""Throughput of the SHAC hot path on one GPU: forward + adjoint window of the 21-hinge
humanoid, 1024 envs, h = 32 frames, 48 substeps per frame (checkpoint every k substeps).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--k 4] [--no-cpu-baseline]
                    [--no-parity] [--no-plain] [--no-theta] [--copy-probe]
    SHACSIM_LIB=phase python bench.py --phase-profile [--model humanoid] [--path persistent|tape]

Prints one JSON line.  A step is one sim_forward_window + sim_adjoint_window pair over
one batch of synthetic inputs already resident in HBM.  Beside the headline number the
line carries: the plain per-substep launch path on the same batch and its speedup, the
policy-parameter gradient pass (timed apart, not part of the step), the FP32 gradient
error against the FP64 kernels together with the FP32 sensitivity floor of the window,
and the FP64 oracle timed on the host.  --copy-probe only runs a device copy of known
size (the calibration of the HBM byte counters).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s fwd+adjoint (h=32), 21-DOF humanoid ×1024 envs; grad err vs FP64"

# MI355X figures used for the roofline (per GPU): AMD's published FP32 vector peak (packed
# FP32, 157.3 TFLOP/s); the same units without packed instructions give half of it, which is
# reported beside it (this build does not emit packed FP32)
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
FP32_VALU_PEAK_TFLOPS = 157.3
FP32_VALU_NONPACKED_TFLOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * 2 * CLOCK_GHZ / 1e3
HBM_PEAK_GBS = 8000.0
# Operations of the FP64 oracle per humanoid env-step (forward window, reverse-mode pass),
# counted at the dispatcher by oracle/count_ops.py (re-derived by tests/test_oracle_count.py).
# The oracle builds the mass matrix and bias in their dense defining form, so these exceed
# the recursive algorithm's count below; they are reported as context, not as the roofline.
ORACLE_OPS_PER_ENV_STEP = {"forward": 9205415, "reverse": 23383710}
# Algorithmic operations of the humanoid, counted by the same counter on the oracle's
# recursive form of the dynamics (oracle/recursive.py, equal to the defining form to
# rounding; re-derived by tests/test_oracle_count.py): one substep (kinematics, contacts,
# recursive Newton-Euler bias, composite-rigid-body mass matrix, Cholesky and solve,
# integration) and its implicit-function adjoint (integrator reverse, the two triangular
# solves of lambda, inverse dynamics at the solved accelerations and its vector-Jacobian
# product), and the per-frame work around them (observation, actor MLP, squash, reward, and
# their reverse with the actor's input VJP).  Recomputation from checkpoints is not counted.
ALGO_OPS = {"substep_forward": 27116, "substep_reverse": 28937, "frame_forward": 111285, "frame_reverse": 112118}
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_window_kernels_humanoid1024_k4.json")
PLAIN_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_plain_kernels_humanoid1024.json")


def kernel_source_hash():
    """SHA-256 over the kernel sources and the C-ABI header (relative path + code, sorted),
    with comments and blank lines removed, so that only code changes invalidate a record."""
    import glob
    import hashlib
    import re
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2204_07137_amd", "csrc", "*.h"))
                   + glob.glob(os.path.join(ROOT, "paper_2204_07137_amd", "csrc", "*.hip"))
                   + glob.glob(os.path.join(ROOT, "include", "*.h")))
    h = hashlib.sha256()
    for f in files:
        with open(f) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = [re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines()]
        h.update(os.path.relpath(f, ROOT).encode())
        h.update("\n".join(line for line in code if line.strip()).encode())
    return h.hexdigest()


def traffic_record(path):
    """A profiler traffic record (FETCH_SIZE / WRITE_SIZE passes scaled by the copy-kernel
    calibration), or None when it is missing or the kernel sources have changed since the
    counters were taken."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    return rec if rec.get("source_sha256") == kernel_source_hash() else None


def adjoint_traffic(n_envs, k, fc):
    """HBM bytes per k_window_adj launch at the headline workload, or None."""
    rec = traffic_record(TRAFFIC_RECORD)
    if rec is None or n_envs != 1024 or k != 4 or bool(rec.get("factor_cache", False)) != fc:
        return None
    return float(rec["bytes_per_launch"])


def mlp_flops(dims):
    return float(sum(2 * a * b for a, b in zip(dims[:-1], dims[1:])))


def algorithmic_bytes(md, n_envs, h, k, actor_dims, elem=4, fc=False):
    """HBM bytes per env-step that the checkpointed window must move: per frame the
    observation, action, reward and dL/da; the checkpoints (S / k states of q, qd) written by
    the forward and read by the adjoint; the actor's hidden activations written by the forward
    and read by the adjoint; with the factor cache, every substep's factor (lower triangle),
    reciprocal pivots, flag and accelerations, written and read; s0, s_h, dL/ds0 and the
    terminal observation once per window."""
    S = int(md["substeps"])
    nq, nv, na = int(md["nq"]), int(md["nv"]), int(md["na"])
    od = actor_dims[0]
    ns = nq + nv + (na if md["has_last_action"] else 0)
    hid = sum(actor_dims[1:-1])
    per_frame = (od + 2 * na + 1) + 2 * (S // k) * (nq + nv) + 2 * hid
    if fc:
        per_frame += 2 * S * (nv * (nv + 1) // 2 + 2 * nv + 1)
    per_window = 3 * ns + od
    return {"per_env_step": elem * (per_frame + per_window / h),
            "what": f"obs + action + reward + dL/da, {S // k} checkpoints written and read, hidden "
                    f"activations written and read" + (", the cached factor and accelerations of "
                    f"{S} substeps written and read" if fc else "") +
                    ", per frame; s0, s_h, dL/ds0, o_h per window (FP32)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--no-factor-cache", action="store_true",
                    help="headline without the factor cache (the adjoint recomputes whole substeps)")
    ap.add_argument("--envs", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the tape / k-sweep / plain comparisons")
    ap.add_argument("--no-theta", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-morphology batch")
    ap.add_argument("--no-mtu", action="store_true", help="skip the muscle-driven humanoid")
    ap.add_argument("--no-long", action="store_true", help="skip the long-window (h up to 256) section")
    ap.add_argument("--no-stoch", action="store_true", help="skip the stochastic-policy window")
    ap.add_argument("--no-term", action="store_true", help="skip the window with early termination")
    ap.add_argument("--no-learn", action="store_true", help="skip the learning-episode section")
    ap.add_argument("--phase-profile", action="store_true",
                    help="only the per-phase cycles of the window kernels (run with SHACSIM_LIB=phase after "
                         "python -m paper_2204_07137_amd.build --phase-profile)")
    ap.add_argument("--model", default="humanoid",
                    help="workload of --phase-profile (mtu: the muscle humanoid's own 2048 envs, k = 16, BF16 MLPs)")
    ap.add_argument("--path", default="persistent", choices=("persistent", "tape"), help="launch form of --phase-profile")
    return ap.parse_args()


def phase_profile(args):
    """Shader-clock cycles per environment and substep of every phase of the forward and the
    adjoint window kernels (the library's phase marks), one window after a warm-up, with the
    kernels' event times for comparison (cycles at the measured clock)."""
    import torch
    import workloads as wl
    import paper_2204_07137_amd as P
    mtu = args.model == "mtu"
    W = wl.workload(args.model) if mtu else wl.workload(args.model, args.envs)
    md, od, h = W["model"], W["obs_dim"], W["h"]
    n_envs = W["n_envs"] if mtu else args.envs
    S = int(md["substeps"])
    k = 16 if mtu else args.k
    kw = dict(path=P.PATH_TAPE) if args.path == "tape" else dict(ckpt_interval=k,
                                                                  factor_cache=not (args.no_factor_cache or mtu))
    if mtu:
        kw["mlp_precision"] = "bf16"
    sim = P.Sim(md, n_envs, h, [od] + [w.shape[0] for w, _ in W["actor"]],
                [od] + [w.shape[0] for w, _ in W["critic"]], **kw)
    s0, actor, critic = sim._dev(W["s0"]), sim.weights(W["actor"]), sim.weights(W["critic"])
    fw = sim.forward(s0, actor, critic)
    sim.adjoint(fw)
    torch.cuda.synchronize()
    P.phase_profile(reset=True)
    out = {"workload": f"{args.model} {n_envs} envs, h={h}, S={S}, {args.path}" +
                       (f" k={k}" + ("" if kw.get("factor_cache") is False else ", factor cache")
                        if args.path == "persistent" else "") + (", BF16 MLPs" if mtu else ""),
           "unit": "shader-clock cycles per env and substep (sum over the env's wavefront time)"}
    env_sub = n_envs * h * S
    for name, run in (("forward", lambda: sim.forward(s0, actor, critic)), ("adjoint", lambda: sim.adjoint(fw))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = run()
        e1.record()
        torch.cuda.synchronize()
        if name == "forward":
            fw = r
        cyc = P.phase_profile(reset=True)
        per = {k: round(v / env_sub, 1) for k, v in cyc.items() if v}
        out[name] = {"ms": round(e0.elapsed_time(e1), 3), "total": round(sum(cyc.values()) / env_sub, 1),
                     "phases": per}
    print(json.dumps(out), flush=True)


def copy_probe():
    """A 256 MiB device-to-device copy, five times: the reference kernel for scaling the
    profiler's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}),
          flush=True)


def time_windows(sim, s0, actor, critic, steps, warmup, want_theta=False, noise=None, log_std=None,
                 reset_states=None):
    """Forward + adjoint windows; per-launch HIP-event times on torch's current stream
    (the stream the window kernels are launched on) and the wall time of the timed loop.
    noise / log_std select the stochastic policy; reset_states early termination."""
    import torch
    for _ in range(warmup):
        fw = sim.forward(s0, actor, critic, noise=noise, log_std=log_std, reset_states=reset_states)
        sim.adjoint(fw, want_theta=want_theta)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        fw = sim.forward(s0, actor, critic, noise=noise, log_std=log_std, reset_states=reset_states)
        ev[i][1].record()
        ad = sim.adjoint(fw, want_theta=want_theta)
        ev[i][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
    adj_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
    return wall, fwd_ms, adj_ms, fw, ad


def mtu_window(P, wl, torch, steps=3):
    """Muscle-driven humanoid: 2048 envs, 152 muscle-tendon units, h = 32, S = 48, FP32
    dynamics with the actor (280-400-200-152) and critic (280-400-200-1) on the BF16
    matrix cores, persistent path with k = 16; gradient error against the FP64 kernels
    (FP64 dynamics and MLPs) reported, not gated."""
    W = wl.workload("mtu")
    N, h = W["n_envs"], W["h"]
    od = W["obs_dim"]
    ad_ = [od] + [w.shape[0] for w, _ in W["actor"]]
    cd_ = [od] + [w.shape[0] for w, _ in W["critic"]]
    sim = P.Sim(W["model"], N, h, ad_, cd_, ckpt_interval=16, mlp_precision="bf16")
    s0 = sim._dev(W["s0"])
    actor, critic = sim.weights(W["actor"]), sim.weights(W["critic"])
    wall, fwd_ms, adj_ms, fw, ad = time_windows(sim, s0, actor, critic, steps, 1)
    # the same window on the tape path (no recomputation in the adjoint)
    st = P.Sim(W["model"], N, h, ad_, cd_, path=P.PATH_TAPE, mlp_precision="bf16")
    twall, tfwd, tadj, _, _ = time_windows(st, s0, actor, critic, steps, 1)
    tape = {"value": round(N * h / (twall / steps), 1), "fwd_ms": round(float(np.mean(tfwd)), 3),
            "adj_ms": round(float(np.mean(tadj)), 3), "workspace_gb": round(st.ws_bytes / 1e9, 2)}
    st.close()
    sim64 = P.Sim(W["model"], N, h, ad_, cd_, ckpt_interval=16, precision="fp64")
    fw64 = sim64.forward(W["s0"], W["actor"], W["critic"])
    ad64 = sim64.adjoint(fw64)
    torch.cuda.synchronize()
    return {"workload": f"muscle humanoid, 152 MTUs, {N} envs, h={h}, S=48, k=16, BF16 MFMA actor/critic",
            "value": round(N * h / (wall / steps), 1), "unit": "env-steps/s",
            "fwd_ms": round(float(np.mean(fwd_ms)), 3), "adj_ms": round(float(np.mean(adj_ms)), 3),
            "workspace_gb": round(sim.ws_bytes / 1e9, 2), "tape_path": tape,
            "err_vs_fp64": {"dL_da": grad_err(ad["dL_da"], ad64["dL_da"], 1),
                            "dL_ds0": grad_err(ad["dL_ds0"], ad64["dL_ds0"], 0),
                            "actions_t0_relmax": float(((fw["actions"][0].double() - fw64["actions"][0]).abs().max()
                                                        / fw64["actions"][0].abs().max()))}}


def mixed_batch(P, wl, torch, budget_gb=64.0, steps=3):
    """Mixed-morphology batch: 4096 CartPole + 2048 Ant + 1024 Humanoid + 512 muscle
    humanoid envs, h = 32.  Each model's launch configuration is picked by the autotuner
    within a shared workspace budget, then all four go out as one graph-captured group
    launch; compared with per-model launches of the plain per-substep path (the muscle
    model, which has no plain path, with its own persistent launch)."""
    members = [("humanoid", 1024), ("mtu", 512), ("ant", 2048), ("cartpole", 4096)]
    Ws, dims = [], []
    for name, n in members:
        W = wl.workload(name, n)
        od = W["obs_dim"]
        Ws.append(W)
        dims.append(([od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]]))
    h = Ws[0]["h"]
    left = budget_gb * 1e9
    tuned, sims, args, costs = [], [], [], []
    for (name, n), W, (ad_, cd_) in zip(members, Ws, dims):
        r = P.tune(W["model"], n, h, ad_, cd_, W["s0"], W["actor"], W["critic"], budget_bytes=int(left), reps=1)
        left -= r["workspace_bytes"]
        kw = dict(path=P.PATH_TAPE) if r["path"] == P.PATH_TAPE else dict(ckpt_interval=r["ckpt_interval"])
        sim = P.Sim(W["model"], n, h, ad_, cd_, lanes_per_env=r["lanes_per_env"],
                    factor_cache=bool(r["factor_cache"]), **kw)
        tuned.append({"model": name, "envs": n, "path": "tape" if r["path"] == P.PATH_TAPE else "persistent",
                      "k": r["ckpt_interval"], "lanes_per_env": r["lanes_per_env"],
                      "factor_cache": bool(r["factor_cache"]),
                      "candidates": r["n_candidates"], "ms_window": round(r["ms_window"], 3),
                      "env_steps_per_s": round(n * h / (r["ms_window"] / 1e3), 1),
                      "workspace_gb": round(r["workspace_bytes"] / 1e9, 2)})
        sims.append(sim)
        args.append((sim._dev(W["s0"]), sim.weights(W["actor"]), sim.weights(W["critic"])))
        costs.append(r["ms_window"] / n)
    G = P.Group(sims, cost_hint=costs)
    total_envs = sum(n for _, n in members)

    def run_group():
        fws = G.forward(args)
        G.adjoint(fws)

    def run_plain(plains):
        for sim, a in zip(plains, args):
            fw = sim.forward(*a)
            sim.adjoint(fw)

    run_group()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_group()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / steps
    plains = [P.Sim(W["model"], n, h, ad_, cd_,
                    **(dict(ckpt_interval=16) if name == "mtu" else dict(path=P.PATH_PLAIN)))
              for (name, n), W, (ad_, cd_) in zip(members, Ws, dims)]
    run_plain(plains)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_plain(plains)
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / steps
    order = [members[i][0] for i in G.order()]
    return {"workload": "4096 cartpole + 2048 ant + 1024 humanoid + 512 muscle-humanoid envs, h=32, one "
                        "graph-captured group launch per direction (autotuned path / k / lanes per env per "
                        "model, 64 GB workspace budget)",
            "value": round(total_envs * h / tg, 1), "unit": "env-steps/s", "ms_per_step": round(tg * 1e3, 3),
            "dispatch_order": order, "tuned": tuned, "graph_captures": G.captures(),
            "plain_per_model": {"value": round(total_envs * h / tp, 1), "ms_per_step": round(tp * 1e3, 3)},
            "speedup_vs_plain": round(tp / tg, 3)}


def grad_err(a, b, per_env_axis=None, envs=None):
    """Relative-norm error and cosine of a against b (flattened), plus the median and
    worst per-env cosine when per_env_axis names the env axis."""
    a64 = a.double()
    b64 = b.double()
    fa, fb = a64.flatten(), b64.flatten()
    out = {"relnorm": float((fa - fb).norm() / fb.norm()),
           "cos": float((fa @ fb) / (fa.norm() * fb.norm()))}
    if per_env_axis is not None:
        A = a64.movedim(per_env_axis, 0).reshape(a64.shape[per_env_axis], -1)
        B = b64.movedim(per_env_axis, 0).reshape(b64.shape[per_env_axis], -1)
        c = (A * B).sum(1) / (A.norm(dim=1) * B.norm(dim=1)).clamp_min(1e-300)
        out["cos_env_median"] = float(c.median())
        out["cos_env_min"] = float(c.min())
        r = (A - B).norm(dim=1) / B.norm(dim=1).clamp_min(1e-300)
        out["rel_env_median"] = float(r.median())
        if envs is not None:
            out["rel_env_median_sampled"] = float(r[list(envs)].median())
    return out


def fp32_storage_floor(h):
    """The oracle's FP32 storage floor of the humanoid window on the 8 sampled envs of the
    headline batch (tests/golden/fp32_floor.json, written by the oracle alone): per-env relative
    error of dL/da and dL/ds0 of the FP64 window whose state, inputs and actions are stored in
    float32, against the plain FP64 window."""
    with open(os.path.join(ROOT, "tests", "golden", "fp32_floor.json")) as fh:
        rec = json.load(fh)["humanoid"]
    row = next((r for r in rec["rows"] if r["h"] == h), None)
    if row is None:
        return None
    return {"what": "oracle FP64 window with float32 storage of state, inputs and actions vs plain FP64, "
                    "8 sampled envs (tests/golden/fp32_floor.json)", "envs": rec["envs"], "h": h,
            "dL_da_rel_env_median": float(np.median([e["dL_da_rel"] for e in row["per_env"]])),
            "dL_ds0_rel_env_median": float(np.median([e["dL_ds0_rel"] for e in row["per_env"]])),
            "h_gate": rec["h_gate"]}


def long_windows(P, wl, torch, n_envs=256, horizons=(32, 64, 128, 256)):
    """BPTT-style long windows of the humanoid (checkpointed, k = 16): FP32 throughput and
    workspace, and the norms of the policy-parameter gradient and of dL/ds0 as the horizon
    grows, from the FP64 kernels (FP32 overflows once they pass ~1e38)."""
    W = wl.workload("humanoid", n_envs)
    md = W["model"]
    od = W["obs_dim"]
    dims = ([od] + [w.shape[0] for w, _ in W["actor"]], [od] + [w.shape[0] for w, _ in W["critic"]])

    def norm(x):
        v = float(x.double().norm())
        return v if np.isfinite(v) else "non-finite"

    res = []
    for h in horizons:
        row = {"h": h}
        for prec in ("fp32", "fp64"):
            sim = P.Sim(md, n_envs, h, dims[0], dims[1], ckpt_interval=16, policy_grad=True, precision=prec)
            s0 = sim._dev(W["s0"])
            actor, critic = sim.weights(W["actor"]), sim.weights(W["critic"])
            wall, _, _, fw, ad = time_windows(sim, s0, actor, critic, 1, 1, want_theta=True)
            if prec == "fp32":
                row["env_steps_per_s"] = round(n_envs * h / wall, 1)
                row["workspace_gb"] = round(sim.ws_bytes / 1e9, 3)
                row["fp32_grad_theta_norm"] = norm(ad["dL_dtheta_flat"])
            else:
                row["grad_theta_norm"] = norm(ad["dL_dtheta_flat"])
                row["grad_s0_norm"] = norm(ad["dL_ds0"])
                row["envs_nonfinite_state"] = int(fw["nonfinite"].sum())
                finite_env = torch.isfinite(ad["dL_ds0"]).all(1)
                row["grad_s0_norm_finite_envs"] = norm(ad["dL_ds0"][finite_env])
                row["envs_nonfinite_grad"] = int((~finite_env).sum())
            sim.close()
        res.append(row)
    return {"workload": f"humanoid {n_envs} envs, k=16, policy-parameter gradient; norms from the FP64 "
                        f"kernels, throughput in FP32", "windows": res}


def learning_episode(P, torch, sim, W, steps=3):
    """SHAC learning episodes on the headline batch (Sec. 3.3, Algorithm "SHAC"; App. A.2
    hyperparameters): the window with the policy-parameter gradient, one Adam step of the
    actor, the target critic's values of the window's states, TD-lambda estimates, the critic
    fit (16 passes x 4 minibatches, Adam), the target-critic update, and the merge of the
    window's observations into the running statistics that normalise the networks' inputs
    in the next episode.  Both learning rates decay linearly to zero over MAX_EPISODES
    (App. A.2: actor 2e-3, critic 5e-4).  The start states are the same every episode (a
    fixed benchmark batch)."""
    MAX_EPISODES = 2000
    N, h, od = sim.N, sim.H, sim.od
    s0 = sim._dev(W["s0"])
    actor = [(a.clone(), b.clone()) for a, b in sim.weights(W["actor"])]
    critic = [(a.clone(), b.clone()) for a, b in sim.weights(W["critic"])]
    target = [(a.clone(), b.clone()) for a, b in critic]
    flat = lambda L: [x for pair in L for x in pair]
    n_a, n_c = sum(x.numel() for x in flat(actor)), sum(x.numel() for x in flat(critic))
    am, av = torch.zeros(n_a, device="cuda"), torch.zeros(n_a, device="cuda")
    cm, cv = torch.zeros(n_c, device="cuda"), torch.zeros(n_c, device="cuda")
    g = torch.Generator().manual_seed(3)
    perm = torch.stack([torch.randperm(h * N, generator=g) for _ in range(16)]).to(torch.int32).cuda()
    ws = sim.critic_workspace((h + 1) * N)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps + 1)]
    mean, var = torch.zeros(od, device="cuda"), torch.ones(od, device="cuda")
    inv = torch.ones(od, device="cuda")
    count = [0]

    def episode(i, e):
        e[0].record()
        fw = sim.forward(s0, actor, target, obs_norm=(mean, inv))
        ad = sim.adjoint(fw, want_theta=True)
        e[1].record()
        decay = max(1.0 - i / MAX_EPISODES, 0.0)
        P.adam_step(flat(actor), ad["dL_dtheta_flat"], am, av, i + 1, 2e-3 * decay)
        vals = sim.critic_values(fw["obs"], target, workspace=ws, obs_norm=(mean, inv)).reshape(h + 1, N)
        tgt = P.td_lambda(fw["rewards"], vals, 0.99, 0.95).reshape(-1)
        sim.critic_fit(fw["obs"][:h].reshape(-1, od), tgt, perm, 4, critic, cm, cv, i * 64, 5e-4 * decay,
                       workspace=ws, obs_norm=(mean, inv))
        P.soft_update(flat(target), flat(critic), 0.995)
        count[0] = P.obs_stats_update(fw["obs"][:h], count[0], mean, var, inv)
        e[2].record()

    episode(0, ev[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        episode(i + 1, ev[i + 1])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    upd = float(np.mean([a[1].elapsed_time(a[2]) for a in ev[1:]]))
    win = float(np.mean([a[0].elapsed_time(a[1]) for a in ev[1:]]))
    return {"workload": f"humanoid {N} envs, h={h}: window + policy gradient + actor Adam + TD-lambda + "
                        f"critic fit 16 x 4 minibatches of {h * N // 4} rows + target update + "
                        f"observation statistics",
            "ms_per_episode": round(wall * 1e3, 3), "episodes_per_s": round(1.0 / wall, 2),
            "env_steps_per_s": round(N * h / wall, 1), "window_ms": round(win, 3), "update_ms": round(upd, 3)}


def fd_directions(sim64, W, ad64, h, n_dirs=8):
    """Central differences of the full FP64 window loss along one random direction per
    sampled env (8 envs, indices from seed 4; positions and velocities, root quaternion
    fixed) against the adjoint's directional derivative, at eps 1e-3 and 1e-6: reported,
    not gated (the contact-rich h = 32 window is far from linear on these scales)."""
    import torch
    md, N = W["model"], sim64.N
    g = sim64.opt.gamma
    rng = np.random.default_rng(4)
    envs = np.sort(rng.choice(N, n_dirs, replace=False))
    ns = W["s0"].shape[1]
    U = np.zeros((N, ns))
    for e in envs:
        u = rng.standard_normal(ns)
        u[3:7] = 0.0
        u[md["nq"] + md["nv"]:] = 0.0
        U[e] = u / np.linalg.norm(u)
    want = (ad64["dL_ds0"].cpu().numpy() * U).sum(1)[envs]

    def env_losses(s0):
        f = sim64.forward(s0, W["actor"], W["critic"])
        torch.cuda.synchronize()
        r, v = f["rewards"].cpu().numpy(), f["value"].cpu().numpy()
        return -(sum(g ** t * r[t] for t in range(h)) + g ** h * v) / (N * h)
    res = {"envs": [int(e) for e in envs], "h": h}
    for eps in (1e-3, 1e-6):
        fd = ((env_losses(W["s0"] + eps * U) - env_losses(W["s0"] - eps * U)) / (2 * eps))[envs]
        rel = np.abs(fd - want) / np.maximum(np.abs(want), 1e-300)
        res[f"eps_{eps:g}"] = {"median_rel_err": float(np.median(rel)), "max_rel_err": float(rel.max())}
    return res


def cpu_baseline(W, h_sample=16, n_envs_sample=64):
    """The FP64 oracle (CPU, PyTorch) on a bounded sample of the same workload: n_envs_sample
    envs of the headline batch over h_sample frames, forward and reverse, scaled to env-steps
    per second (the oracle's cost is linear in frames; envs run as one batch).  cores is the
    process's CPU time over the wall time of the run: the threads it kept busy."""
    import torch
    from oracle import oracle_window_grads
    t0, c0 = time.time(), time.process_time()
    oracle_window_grads(W["model"], W["s0"][:n_envs_sample], h_sample, W["actor"], W["critic"],
                        n_total=W["n_envs"])
    dt, dc = time.time() - t0, time.process_time() - c0
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n_envs_sample * h_sample / dt, "unit": "env-steps/s", "cores": round(dc / dt, 1),
            "kind": "oracle", "cpu": cpu, "nproc": os.cpu_count(), "torch_threads": torch.get_num_threads(),
            "sample": f"{n_envs_sample} humanoid envs of the headline batch x h={h_sample} frames (48 substeps "
                      f"each), fwd+reverse, {dt:.1f} s wall; env-steps/s of the sample (the oracle's cost "
                      f"is linear in frames)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the envs are "
              f"independent and would shard with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as wl
    import paper_2204_07137_amd as P

    torch.manual_seed(0)
    if args.copy_probe:
        copy_probe()
        return
    if args.phase_profile:
        phase_profile(args)
        return
    W = wl.workload("humanoid", args.envs)
    md = W["model"]
    od = W["obs_dim"]
    h = W["h"]
    S = int(md["substeps"])
    actor_dims = [od] + [w.shape[0] for w, _ in W["actor"]]
    critic_dims = [od] + [w.shape[0] for w, _ in W["critic"]]
    N = args.envs
    fc = not args.no_factor_cache
    sim = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=args.k, policy_grad=not args.no_theta,
                factor_cache=fc)
    s0 = sim._dev(W["s0"])
    actor = sim.weights(W["actor"])
    critic = sim.weights(W["critic"])
    wall, fwd_ms, adj_ms, fw, ad = time_windows(sim, s0, actor, critic, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    value = N * h / (wall / args.steps)

    # roofline of the dominant kernel (the adjoint window kernel): counted algorithmic
    # operations (ALGO_OPS) per env-step, without the recomputation of the forward
    adj_flops_env_step = S * ALGO_OPS["substep_reverse"] + ALGO_OPS["frame_reverse"]
    fwd_flops_env_step = S * ALGO_OPS["substep_forward"] + ALGO_OPS["frame_forward"]
    adj_launch_flops = adj_flops_env_step * N * h
    adj_avg_s = float(np.mean(adj_ms)) / 1e3
    fwd_avg_s = float(np.mean(fwd_ms)) / 1e3
    achieved = adj_launch_flops / adj_avg_s / 1e12
    fwd_achieved = fwd_flops_env_step * N * h / fwd_avg_s / 1e12
    hbm = algorithmic_bytes(md, N, h, args.k, actor_dims, fc=fc)
    step_s = wall / args.steps
    roof = {"bound": "alu", "kernel": "k_window_adj", "achieved": round(achieved, 4),
            "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VALU_PEAK_TFLOPS, 5), "traffic": adjoint_traffic(N, args.k, fc),
            "traffic_unit": "bytes per launch, profiler FETCH_SIZE + WRITE_SIZE scaled by a copy of known size",
            "flops_per_env_step": {"adjoint_kernel": adj_flops_env_step, "forward_kernel": fwd_flops_env_step,
                                   "counted": "oracle recursive form (oracle/count_ops.py), no recompute"},
            "frac_of_nonpacked_peak": round(achieved / FP32_VALU_NONPACKED_TFLOPS, 5),
            "nonpacked_peak": round(FP32_VALU_NONPACKED_TFLOPS, 1),
            "forward_kernel": {"achieved": round(fwd_achieved, 4), "frac": round(fwd_achieved / FP32_VALU_PEAK_TFLOPS, 5)},
            "oracle_ops_per_env_step": ORACLE_OPS_PER_ENV_STEP,
            "avg_ms": {"k_window_adj": round(float(np.mean(adj_ms)), 3),
                       "k_window_fwd": round(float(np.mean(fwd_ms)), 3)}}
    # HBM: the window's algorithmic bytes over the step, and the adjoint kernel's counted bytes
    hbm_out = {"algorithmic_bytes_per_env_step": hbm["per_env_step"], "what": hbm["what"],
               "algorithmic_gbs": round(hbm["per_env_step"] * N * h / step_s / 1e9, 2),
               "algorithmic_frac": round(hbm["per_env_step"] * N * h / step_s / 1e9 / HBM_PEAK_GBS, 6)}
    if roof["traffic"] is not None:
        hbm_out["adjoint_counter_gbs"] = round(roof["traffic"] / adj_avg_s / 1e9, 1)
        hbm_out["adjoint_counter_frac"] = round(roof["traffic"] / adj_avg_s / 1e9 / HBM_PEAK_GBS, 4)
    roof["hbm"] = hbm_out

    n_eval = N * h * S * len(md["contact_body"])
    contacts = {"adhesive_frac": round(float(fw["adhesive_count"].double().sum()) / n_eval, 6),
                "evaluations": n_eval,
                "what": "contact evaluations (envs x frames x substeps x contacts) whose literal "
                        "normal force pulls (d < 0, d_dot > k_n / k_d)"}
    out = {"metric": METRIC, "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"humanoid 13 bodies / 21 hinges / 10 contacts, {N} envs, h={h}, "
                                  f"S={S} substeps, checkpoint k={args.k}"
                                  f"{', cached factorisation' if fc else ''}, actor 76-256-128-21, "
                                  f"critic 76-128-128-1", "envs": N, "h": h, "substeps": S,
                      "ckpt_interval": args.k, "path": "persistent", "factor_cache": fc,
                      "workspace_gb": round(sim.ws_bytes / 1e9, 3)},
           "roofline": roof, "contacts": contacts,
           # the paper's own figures (App. A.4, wall-clock breakdown of a training episode),
           # context only: another GPU, 64 envs, and its backward includes the actor update
           "paper_context": {"humanoid_env_steps_per_s": 711, "muscle_humanoid_env_steps_per_s": 826,
                             "derived_as": "64 envs x 32 steps / (forward + backward seconds)",
                             "hardware": "NVIDIA TITAN X, Intel Xeon E5-2620", "precision": "not stated"}}

    if not args.no_theta:
        # policy-parameter gradient pass: adjoint with and without it, the difference
        _, _, adj_th_ms, _, _ = time_windows(sim, s0, actor, critic, max(3, args.steps // 4), 1,
                                             want_theta=True)
        th_ms = max(float(np.median(adj_th_ms)) - float(np.median(adj_ms)), 0.0)
        rows = N * h
        # the contractions the pass runs: every layer's weight gradient and the input adjoints
        # of layers 1.. (the hidden activations are the window's own, FP32 networks)
        layer = [a * b for a, b in zip(actor_dims[:-1], actor_dims[1:])]
        th_flops = 2 * rows * (sum(layer) + sum(layer[1:]))
        out["policy_grad"] = {"ms": round(th_ms, 3), "rows": rows,
                              "mfma_tflops": round(th_flops / max(th_ms, 1e-6) / 1e9, 3),
                              "mfma_peak_fp32_tflops": 157.3}

    if not args.no_stoch:
        # the same window under the stochastic policy (reparameterised Gaussian, draws as inputs)
        rng = np.random.default_rng(7)
        noise = torch.as_tensor(rng.standard_normal((h, N, md["na"])), dtype=torch.float32, device="cuda")
        log_std = torch.full((md["na"],), -1.0, dtype=torch.float32, device="cuda")
        sw, _, _, _, _ = time_windows(sim, s0, actor, critic, max(3, args.steps // 4), 1, noise=noise,
                                      log_std=log_std)
        sval = N * h / (sw / max(3, args.steps // 4))
        out["stochastic_policy"] = {"value": round(sval, 1), "unit": "env-steps/s", "log_std": -1.0,
                                    "vs_deterministic": round(sval / value, 3)}

    if not args.no_term:
        # the same window with early termination at the humanoid's torso height (0.74 m):
        # per-frame test, reset from per-env restart states, discount and gradient cut
        mdt = wl.with_termination(md)
        simt = P.Sim(mdt, N, h, actor_dims, critic_dims, ckpt_interval=args.k, factor_cache=fc)
        reset = simt._dev(wl.initial_states(mdt, N, seed=9))
        n_t = max(3, args.steps // 4)
        tw, _, _, tfw, _ = time_windows(simt, s0, actor, critic, n_t, 1, reset_states=reset)
        tval = N * h / (tw / n_t)
        done = tfw["done"].float()
        out["early_termination"] = {"value": round(tval, 1), "unit": "env-steps/s",
                                    "term_height_m": float(mdt["term_height"]),
                                    "done_frac_per_frame": round(float(done.mean()), 4),
                                    "envs_terminated": int((done.sum(0) > 0).sum()),
                                    "vs_no_termination": round(tval / value, 3)}
        simt.close()

    if not args.no_plain:
        # the same window on the other launch forms: the tape path (the forward records
        # every substep's linearisation, the adjoint recomputes nothing), the other
        # checkpoint intervals, and the plain per-substep launch path
        tape = P.Sim(md, N, h, actor_dims, critic_dims, path=P.PATH_TAPE)
        tw, tf, ta, _, _ = time_windows(tape, s0, actor, critic, max(3, args.steps // 4), 1)
        tval = N * h / (tw / max(3, args.steps // 4))
        out["tape_path"] = {"value": round(tval, 1), "unit": "env-steps/s",
                            "fwd_ms": round(float(np.mean(tf)), 3), "adj_ms": round(float(np.mean(ta)), 3),
                            "workspace_gb": round(tape.ws_bytes / 1e9, 2),
                            "vs_persistent": round(tval / value, 3)}
        del tape
        # the same checkpoint interval with the other factor-cache setting
        so = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=args.k, factor_cache=not fc)
        ow, of, oa, _, _ = time_windows(so, s0, actor, critic, max(3, args.steps // 4), 1)
        oval = N * h / (ow / max(3, args.steps // 4))
        out["recompute_path" if fc else "factor_cache_path"] = {
            "value": round(oval, 1), "unit": "env-steps/s", "factor_cache": not fc,
            "fwd_ms": round(float(np.mean(of)), 3), "adj_ms": round(float(np.mean(oa)), 3),
            "workspace_gb": round(so.ws_bytes / 1e9, 3), "vs_headline": round(oval / value, 3)}
        del so
        sweep = {}
        for kk in (1, 2, 4, 8, 16):
            if kk == args.k:
                sweep[str(kk)] = round(value, 1)
                continue
            sk = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=kk, factor_cache=fc)
            kw, _, _, _, _ = time_windows(sk, s0, actor, critic, 3, 1)
            sweep[str(kk)] = round(N * h / (kw / 3), 1)
            del sk
        out["ckpt_sweep"] = sweep
        plain = P.Sim(md, N, h, actor_dims, critic_dims, path=P.PATH_PLAIN)
        pw, pf, pa, _, _ = time_windows(plain, s0, actor, critic, args.plain_steps, 1)
        pval = N * h / (pw / args.plain_steps)
        out["plain_path"] = {"value": round(pval, 1), "unit": "env-steps/s",
                             "ms_per_step": round(pw * 1e3 / args.plain_steps, 3),
                             "fwd_ms": round(float(np.mean(pf)), 3), "adj_ms": round(float(np.mean(pa)), 3),
                             "launches_per_step": 2 * (h * (S + 1) + 1),
                             "persistent_speedup": round(value / pval, 3),
                             "tape_speedup": round(tval / pval, 3)}
        # the same algorithmic work per window as the persistent path
        plain_flops = (fwd_flops_env_step + adj_flops_env_step) * N * h
        plain_s = pw / args.plain_steps
        out["plain_path"]["achieved_tflops"] = round(plain_flops / plain_s / 1e12, 4)
        out["plain_path"]["frac_fp32_valu"] = round(plain_flops / plain_s / 1e12 / FP32_VALU_PEAK_TFLOPS, 5)
        prec = traffic_record(PLAIN_TRAFFIC_RECORD)
        if prec is not None:
            out["plain_path"]["traffic_bytes_per_step"] = prec["bytes_per_step"]
            out["plain_path"]["hbm_gbs"] = round(prec["bytes_per_step"] / plain_s / 1e9, 1)
            out["plain_path"]["hbm_frac"] = round(prec["bytes_per_step"] / plain_s / 1e9 / HBM_PEAK_GBS, 4)
        del plain

    # measured device ceilings beside the published ones
    ceil = P.probe_ceilings()
    out["ceilings"] = {"measured_fp32_valu_tflops_nonpacked": round(ceil["fp32_valu_tflops"], 2),
                       "published_fp32_valu_tflops": FP32_VALU_PEAK_TFLOPS,
                       "published_fp32_valu_tflops_nonpacked": round(FP32_VALU_NONPACKED_TFLOPS, 1),
                       "measured_copy_gbs": round(ceil["copy_gbs"], 1),
                       "published_hbm_gbs": HBM_PEAK_GBS}
    roof["frac_of_measured"] = round(achieved / ceil["fp32_valu_tflops"], 5)

    if not args.no_theta and not args.no_learn:
        out["learning_episode"] = learning_episode(P, torch, sim, W)
    if not args.no_long:
        out["long_windows"] = long_windows(P, wl, torch)
    if not args.no_mtu:
        out["mtu"] = mtu_window(P, wl, torch)
    if not args.no_mixed:
        out["mixed"] = mixed_batch(P, wl, torch)

    if not args.no_parity:
        # FP32 error against the FP64 instantiation of the same kernels, beside the oracle's
        # FP32 storage floor of the same window on the same sampled envs
        sim64 = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=args.k, precision="fp64")
        fw64 = sim64.forward(W["s0"], W["actor"], W["critic"])
        ad64 = sim64.adjoint(fw64)
        torch.cuda.synchronize()
        floor = fp32_storage_floor(h)
        envs = floor["envs"] if floor else None
        out["grad_err_vs_fp64"] = {"dL_da": grad_err(ad["dL_da"], ad64["dL_da"], 1, envs),
                                   "dL_ds0": grad_err(ad["dL_ds0"], ad64["dL_ds0"], 0, envs),
                                   "s_h_relmax": float(((fw["s_h"].double() - fw64["s_h"]).abs().max()
                                                        / fw64["s_h"].abs().max()))}
        out["fp32_storage_floor"] = floor
        out["fd_directions"] = fd_directions(sim64, W, ad64, h)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
