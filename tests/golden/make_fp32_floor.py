"""Writes fp32_floor.json: the FP32 storage floor of the humanoid and muscle-humanoid
windows, from the FP64 oracle alone.

For each horizon h, the oracle's window is run twice on the same sampled envs: in plain
FP64, and with the FP32 storage floor (inputs, actions and the dynamic state rounded to
float32 after every substep, arithmetic in FP64).  Per env the file records how far the
rounded window's outputs and gradients are from the FP64 ones (cosine and relative norm of
dL/da and dL/ds0, max-norm relative error of s_h).  An FP32 simulator stores its state in
float32, so it cannot be closer to the FP64 window than this, and the largest h at which
every sampled env stays under the parity bar (states 1e-4, gradient cosine 0.999 and relative
norm 1e-3) is the longest window on which an FP32 path can be held to that bar (h_max_under_bar).
An FP32 simulator also rounds every operation, not only the stored state, so the horizon at
which an FP32 path is gated against the FP64 oracle (h_gate) keeps a margin: the longest window
on which twice the floor stays under the bar at every sampled env.  The muscle humanoid's
networks run in BF16 (its configuration), so both of its runs use the oracle's BF16
emulation.

    python tests/golden/make_fp32_floor.py               # 30 minutes on 8 cores
    python tests/golden/make_fp32_floor.py --summarise   # recompute the summary fields only
"""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as wl  # noqa: E402
from oracle import oracle_window_grads  # noqa: E402

BAR = {"state_rel": 1e-4, "grad_cos": 0.999, "grad_rel": 1e-3}
GATE_MARGIN = 2.0


def under_bar(r, margin=1.0):
    """An env's floor errors, scaled by margin, are under the bar."""
    return (margin * r["s_h_rel"] <= BAR["state_rel"]
            and 1.0 - margin * (1.0 - min(r["dL_da_cos"], r["dL_ds0_cos"])) >= BAR["grad_cos"]
            and margin * max(r["dL_da_rel"], r["dL_ds0_rel"]) <= BAR["grad_rel"])


def longest_under(rows, margin):
    """The longest horizon before the first one at which some sampled env leaves the bar."""
    h = 0
    for r in rows:
        if not all(under_bar(e, margin) for e in r["per_env"]):
            break
        h = r["h"]
    return h


def summarise(out):
    for key in ("humanoid", "mtu"):
        rows = out[key]["rows"]
        for r in rows:
            r["all_under_bar"] = all(under_bar(e) for e in r["per_env"])
        out[key]["h_max_under_bar"] = longest_under(rows, 1.0)
        out[key]["gate_margin"] = GATE_MARGIN
        out[key]["h_gate"] = longest_under(rows, GATE_MARGIN)
        print(key, "h_max_under_bar", out[key]["h_max_under_bar"], "h_gate", out[key]["h_gate"], flush=True)
    return out


def _cos(a, b):
    return float((a * b).sum() / np.sqrt((a * a).sum() * (b * b).sum()))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def floor_rows(name, n_total, envs, horizons, bf16=False):
    W = wl.workload(name, n_total)
    rows = []
    for h in horizons:
        t0 = time.time()
        kw = dict(n_total=n_total, bf16=bf16)
        ref = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], **kw)
        fl = oracle_window_grads(W["model"], W["s0"][envs], h, W["actor"], W["critic"], fp32_floor=True, **kw)
        per_env = []
        for i, e in enumerate(envs):
            a, b = fl["dL_da"][:, i], ref["dL_da"][:, i]
            c, d = fl["dL_ds0"][i], ref["dL_ds0"][i]
            sh = float(np.abs(fl["s_h"][i] - ref["s_h"][i]).max() / np.abs(ref["s_h"][i]).max())
            per_env.append({"env": int(e), "dL_da_cos": _cos(a, b), "dL_da_rel": _rel(a, b),
                            "dL_ds0_cos": _cos(c, d), "dL_ds0_rel": _rel(c, d), "s_h_rel": sh})
        under = all(under_bar(r) for r in per_env)
        rows.append({"h": h, "per_env": per_env, "all_under_bar": under})
        print(f"{name} h={h}: {time.time() - t0:.1f} s, under bar: {under}", flush=True)
    return rows


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp32_floor.json")
    if "--summarise" in sys.argv:
        with open(path) as fh:
            out = summarise(json.load(fh))
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        return
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    rng = np.random.default_rng(4)
    hum_envs = [int(e) for e in np.sort(rng.choice(1024, 8, replace=False))]
    mtu_envs = [int(e) for e in np.sort(np.random.default_rng(4).choice(2048, 4, replace=False))]
    out = {"_source": "tests/golden/make_fp32_floor.py (FP64 oracle only)",
           "bar": BAR,
           "humanoid": {"n_envs": 1024, "envs": hum_envs, "env_seed": 4,
                        "rows": floor_rows("humanoid", 1024, hum_envs, [1, 2, 4, 5, 6, 8, 16, 32])},
           "mtu": {"n_envs": 2048, "envs": mtu_envs, "env_seed": 4, "bf16": True,
                   "rows": floor_rows("mtu", 2048, mtu_envs, [1, 2, 4, 8, 16], bf16=True)}}
    summarise(out)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
