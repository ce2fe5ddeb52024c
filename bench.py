"""Throughput of the SHAC hot path on one GPU: forward + adjoint window of the 21-hinge
humanoid, 1024 envs, h = 32 frames, 48 substeps per frame (checkpoint every k substeps).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--k 16] [--no-cpu-baseline]

Prints one JSON line.  A step is one sim_forward_window + sim_adjoint_window pair over
one batch of synthetic inputs already resident in HBM.
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

# MI355X figures used for the roofline (per GPU)
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
FP32_VALU_PEAK_TFLOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * 2 * CLOCK_GHZ / 1e3   # non-packed FMA
HBM_PEAK_GBS = 8000.0


def substep_flops(md):
    """Floating-point operations (FMA = 2) of one forward substep and of one substep
    adjoint of the recursive algorithm, from the model's structure.  Counts per phase:
    kinematics/velocity/bias acceleration per hinge 185 (root 45), contact force 55 per
    sphere, body inertia + Newton-Euler force 245 per frame, subtree sums 16 per edge,
    bias projection and CRBA column 11 + 11 * depth per hinge (root block 36), dense
    Cholesky 2 n^3 / 3, two triangular solves 2 n^2, integration 2 per hinge + 46 root.
    Adjoint: integrator 60, lambda solves 2 n^2, accelerations / virtual velocities 54 per
    hinge, contact adjoints 120 per sphere, per-body products 300 per frame, 42 subtree
    sums per edge, closed-form derivatives 200 per hinge (1800 root), update 50."""
    J = int(md["n_joints"])
    nv = int(md["nv"])
    nc = len(md["contact_body"])
    par = md["parent"]
    depth = np.zeros(J, int)
    for j in range(J):
        depth[j] = 0 if par[j] < 0 else depth[par[j]] + 1
    hinges = [j for j in range(J) if md["jtype"][j] != 0]
    free = J - len(hinges)
    fwd = (185 * len(hinges) + 45 * free + 55 * nc + 245 * J + 16 * (J - 1)
           + sum(11 + 11 * depth[j] for j in hinges) + 36 * free
           + 2 * nv ** 3 / 3 + 2 * nv * nv + 2 * len(hinges) + 46 * free)
    adj = (60 + 2 * nv * nv + 54 * len(hinges) + 120 * nc + 300 * J + 42 * (J - 1)
           + 200 * len(hinges) + 1800 * free + 50)
    return float(fwd), float(adj)


def mlp_flops(dims):
    return float(sum(2 * a * b for a, b in zip(dims[:-1], dims[1:])))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--envs", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    return ap.parse_args()


def cpu_baseline(W, h, n_envs_sample=2):
    """The FP64 oracle (CPU, PyTorch) on a bounded sample of the same workload."""
    import torch
    from oracle import oracle_window_grads
    t0 = time.time()
    oracle_window_grads(W["model"], W["s0"][:n_envs_sample], h, W["actor"], W["critic"],
                        n_total=W["n_envs"])
    dt = time.time() - t0
    return {"value": n_envs_sample * h / dt, "unit": "env-steps/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n_envs_sample} humanoid envs x h={h} frames (48 substeps each), fwd+reverse, "
                      f"{dt:.1f} s wall"}


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
    W = wl.workload("humanoid", args.envs)
    md = W["model"]
    od = W["obs_dim"]
    h = W["h"]
    S = int(md["substeps"])
    actor_dims = [od] + [w.shape[0] for w, _ in W["actor"]]
    critic_dims = [od] + [w.shape[0] for w, _ in W["critic"]]
    N = args.envs
    sim = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=args.k)
    s0 = sim._dev(W["s0"])
    actor = sim.weights(W["actor"])
    critic = sim.weights(W["critic"])
    for _ in range(args.warmup):
        fw = sim.forward(s0, actor, critic)
        sim.adjoint(fw)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        fw = sim.forward(s0, actor, critic)
        ev[i][1].record()
        ad = sim.adjoint(fw)
        ev[i][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
    adj_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
    ms_per_step = wall * 1e3 / args.steps
    value = N * h / (wall / args.steps)

    # roofline of the dominant kernel (the adjoint window kernel)
    f_sub, a_sub = substep_flops(md)
    mlp_a = mlp_flops(actor_dims)
    adj_flops_env_step = S * (f_sub + a_sub) + 2 * mlp_a + mlp_a     # re-linearise + reverse, MLP fwd + VJP
    fwd_flops_env_step = S * f_sub + mlp_a
    adj_launch_flops = adj_flops_env_step * N * h
    adj_avg_s = float(np.mean(adj_ms)) / 1e3
    achieved = adj_launch_flops / adj_avg_s / 1e12
    roof = {"bound": "alu", "kernel": "k_window_adj", "achieved": round(achieved, 4),
            "peak": round(FP32_VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VALU_PEAK_TFLOPS, 5), "traffic": None,
            "flops_per_env_step": {"adjoint_kernel": adj_flops_env_step, "forward_kernel": fwd_flops_env_step},
            "avg_ms": {"k_window_adj": round(float(np.mean(adj_ms)), 3),
                       "k_window_fwd": round(float(np.mean(fwd_ms)), 3)}}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"humanoid 13 bodies / 21 hinges / 10 contacts, {N} envs, h={h}, "
                                  f"S={S} substeps, checkpoint k={args.k}, actor 76-256-128-21, "
                                  f"critic 76-128-128-1", "envs": N, "h": h, "substeps": S,
                      "ckpt_interval": args.k, "path": "persistent"},
           "roofline": roof}

    if not args.no_parity:
        # error of the FP32 gradients against the FP64 instantiation of the same kernels
        sim64 = P.Sim(md, N, h, actor_dims, critic_dims, ckpt_interval=args.k, precision="fp64")
        fw64 = sim64.forward(W["s0"], W["actor"], W["critic"])
        ad64 = sim64.adjoint(fw64)
        torch.cuda.synchronize()

        def err(a, b):
            a = a.double().flatten()
            b = b.double().flatten()
            return {"relnorm": float((a - b).norm() / b.norm()),
                    "cos": float((a @ b) / (a.norm() * b.norm()))}
        out["grad_err_vs_fp64"] = {"dL_da": err(ad["dL_da"], ad64["dL_da"]),
                                   "dL_ds0": err(ad["dL_ds0"], ad64["dL_ds0"]),
                                   "s_h_relmax": float(((fw["s_h"].double() - fw64["s_h"]).abs().max()
                                                        / fw64["s_h"].abs().max()))}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
