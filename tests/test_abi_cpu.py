"""CPU checks of the C ABI: the library loads, exports every declared entry point, and
rejects bad models and options before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2204_07137_amd as P
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "shacsim.h")).read()
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared()
    assert set(names) == set(P.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def _create(md, **kw):
    d, keep = P.model_desc(md)
    o = P.SimOptions()
    o.n_envs = kw.get("n_envs", 4)
    o.horizon = kw.get("horizon", 2)
    o.ckpt_interval = kw.get("k", md["substeps"])
    o.path = kw.get("path", 0)
    o.closed_loop = 0
    od = {"cartpole": 5, "ant": 37, "humanoid": 76}.get(md["task"], 1)
    dims = kw.get("critic", [od, 8, 1])
    o.critic_layers = len(dims) - 1
    for i, v in enumerate(dims):
        o.critic_dims[i] = v
    o.gamma = 0.99
    o.policy_grad = kw.get("policy_grad", 0)
    o.mlp_precision = kw.get("mlp_precision", 0)
    o.precision = kw.get("precision", 0)
    o.lanes_per_env = kw.get("lanes", 0)
    o.factor_cache = kw.get("factor_cache", 0)
    o.layer_norm = kw.get("layer_norm", 0)
    h = ctypes.c_void_p()
    rc = P.lib().sim_create(ctypes.byref(d), ctypes.byref(o), ctypes.byref(h))
    return rc, P.lib().sim_last_error().decode()


def test_null_arguments_rejected():
    L = P.lib()
    assert L.sim_create(None, None, None) == -1
    assert L.sim_workspace_bytes(None) == 0
    assert L.sim_forward_window(None, None, None) == -2
    assert L.sim_adjoint_window(None, None, None) == -2
    L.sim_destroy(None)
    g = ctypes.c_void_p()
    assert L.sim_group_create(None, 2, None, ctypes.byref(g)) == -1
    bogus = (ctypes.c_void_p * 1)(None)
    assert L.sim_group_create(bogus, 1, None, ctypes.byref(g)) == -2
    assert L.sim_group_create(bogus, 0, None, ctypes.byref(g)) == -1
    assert L.sim_group_forward(None, None, None) == -2
    assert L.sim_group_adjoint(None, None, None) == -2
    assert L.sim_group_info(None, None, None) == -2
    L.sim_group_destroy(None)
    assert L.sim_tune(None, None, None, 0, 1, None, None) == -1
    # learning-episode calls: argument errors before any launch
    z = (ctypes.c_void_p * 1)(None)
    n1 = (ctypes.c_size_t * 1)(4)
    assert L.sim_adam_step(None, None, 1, None, None, None, 1, 1e-3, 0.7, 0.95, 1e-8, 0, None) == -1
    assert L.sim_adam_step(z, n1, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1,
                           1e-3, 0.7, 0.95, 1e-8, 0, None) == -1          # null tensor
    assert L.sim_soft_update(None, None, None, 1, 0.5, 0, None) == -1
    assert L.sim_td_lambda(None, None, None, 4, 4, 0.99, 0.95, None, 0, None) == -1
    assert L.sim_td_lambda(ctypes.c_void_p(16), ctypes.c_void_p(16), None, 4, 4, 1.5, 0.95, ctypes.c_void_p(16), 0,
                           None) == -1                                     # gamma outside [0, 1]
    assert L.sim_critic_workspace_bytes(None, 16) == 0
    assert L.sim_critic_values(None, None, 1, None, None, None, None, None, None, 0, None) == -2
    # running observation statistics: argument errors before any launch
    v16 = ctypes.c_void_p(16)
    assert L.sim_obs_stats_update(None, 4, 3, 0.0, v16, v16, v16, 1e-5, 0, None) == -1
    assert L.sim_obs_stats_update(v16, 0, 3, 0.0, v16, v16, v16, 1e-5, 0, None) == -1       # no rows
    assert L.sim_obs_stats_update(v16, 4, 3, -1.0, v16, v16, v16, 1e-5, 0, None) == -1      # negative count
    assert L.sim_obs_stats_update(v16, 4, 3, 0.0, v16, v16, v16, 1e-5, 7, None) == -1       # precision
    assert L.sim_critic_fit(None, None, None) == -2
    # ceiling probes: argument errors before any launch
    d = ctypes.c_double()
    assert L.sim_probe_fma_bytes() > 0
    assert L.sim_probe_fma(None, 0, None, ctypes.byref(d)) == -1
    assert L.sim_probe_fma(ctypes.c_void_p(16), 16, None, ctypes.byref(d)) == -1     # scratch too small
    assert L.sim_probe_copy(None, None, 64, None, ctypes.byref(d)) == -1
    assert L.sim_probe_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), 24, None, ctypes.byref(d)) == -1
    assert L.sim_probe_copy(ctypes.c_void_p(8), ctypes.c_void_p(32), 64, None, ctypes.byref(d)) == -1


def test_model_limits_rejected():
    md = wl.humanoid()
    bad = dict(md)
    bad["parent"] = md["parent"].copy()
    bad["parent"][3] = 5
    rc, msg = _create(bad)
    assert rc == -4 and "parents" in msg
    rc, msg = _create(md, k=5)
    assert rc == -1 and "ckpt_interval" in msg
    rc, msg = _create(md, k=1, path=1)
    assert rc != -1 or "ckpt" not in msg
    rc, msg = _create(md, k=16, path=1)
    assert rc == -1 and "plain" in msg
    rc, msg = _create(md, critic=[75, 8, 1])
    assert rc == -1 and "critic" in msg
    rc, msg = _create(md, policy_grad=1)
    assert rc == -1 and "policy_grad" in msg
    rc, msg = _create(md, policy_grad=2)
    assert rc == -1 and "policy_grad" in msg
    rc, msg = _create(md, mlp_precision=1, precision=1)
    assert rc == -1 and "BF16" in msg
    rc, msg = _create(md, mlp_precision=3)
    assert rc == -1 and "mlp_precision" in msg
    mm = wl.mtu_humanoid()
    rc, msg = _create(mm, path=1, k=1, critic=[280, 8, 1])
    assert rc == -6 and "muscle" in msg


def test_too_many_joints_rejected():
    md = wl.chain(40, free_root=True)
    md["task"] = "none"
    rc, msg = _create(md, critic=[1, 1])
    assert rc == -4 and "n_joints" in msg


def test_termination_model_and_path_checks():
    """Early termination needs a free root and runs on the persistent and tape paths only:
    both are rejected at sim_create, before anything reaches the device."""
    import workloads as wl
    cp = wl.with_termination(dict(wl.workload("cartpole", 4)["model"], et_height=0.5))
    rc, msg = _create(cp)
    assert rc == -4 and "FREE root" in msg
    ant = wl.with_termination(wl.workload("ant", 4)["model"])
    rc, msg = _create(ant, path=1, k=1)
    assert rc == -6 and "persistent and tape" in msg


def _header_members(struct):
    """Member names, in order, of `typedef struct <struct> { ... } <struct>;` in shacsim.h."""
    src = open(os.path.join(ROOT, "include", "shacsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), src, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):           # "double lr, beta1, beta2, eps"
            m = re.search(r"\**\s*([A-Za-z_]\w*)\s*(\[[^\]]*\])*\s*$", part.strip())
            names.append(m.group(1))
    return names


@pytest.mark.parametrize("struct", ["SimModelDesc", "SimOptions", "SimForwardIO", "SimAdjointIO", "SimTuneResult",
                                    "SimCriticFitIO"])
def test_binding_structs_match_the_header(struct):
    """The ctypes structures of the binding declare the C structs' members in the same order
    (a mismatch would shift every later field of a call)."""
    assert [f[0] for f in getattr(P, struct)._fields_] == _header_members(struct)


ABI_IDS = {"SimModelDesc": 0, "SimOptions": 1, "SimForwardIO": 2, "SimAdjointIO": 3, "SimTuneResult": 4,
           "SimCriticFitIO": 5}


@pytest.mark.parametrize("struct", sorted(ABI_IDS))
def test_binding_struct_sizes_and_offsets_match_the_library(struct):
    """Byte size and every member's byte offset of the binding's ctypes structures equal those
    the library was compiled with (sim_abi_layout): a changed member type would move them."""
    L = P.lib()
    cls = getattr(P, struct)
    sid = ABI_IDS[struct]
    assert ctypes.sizeof(cls) == L.sim_abi_layout(sid, -1)
    for i, (name, _) in enumerate(cls._fields_):
        assert getattr(cls, name).offset == L.sim_abi_layout(sid, i), (struct, name)
    assert L.sim_abi_layout(sid, len(cls._fields_)) == ctypes.c_size_t(-1).value
    assert L.sim_abi_layout(99, 0) == ctypes.c_size_t(-1).value


def test_compact_layout_checks():
    """lanes_per_env (the compact layout, several small envs per wavefront) is checked at
    sim_create, before anything reaches the device: lane counts, precision, BF16 networks,
    muscle models, the plain path, models beyond its capacities, and n_envs that do not fill
    whole wavefronts are refused."""
    ant = wl.workload("ant", 4)["model"]
    for lanes, kw, code, text in ((8, {}, -1, "lanes_per_env"),
                                  (16, dict(precision=1), -6, "FP32"),
                                  (16, dict(mlp_precision=1), -6, "FP32 MLPs"),
                                  (16, dict(path=1, k=1), -6, "persistent and tape"),
                                  (16, dict(n_envs=6), -1, "multiple of 64 / lanes_per_env"),
                                  (16, dict(critic=[37, 256, 1]), -6, "critic width")):
        rc, msg = _create(ant, lanes=lanes, **kw)
        assert rc == code and text in msg, (lanes, kw, rc, msg)
    rc, msg = _create(wl.humanoid(), lanes=32, critic=[76, 8, 1])
    assert rc == -6 and "beyond the compact layout" in msg
    mm = wl.mtu_humanoid()
    rc, msg = _create(mm, lanes=64, critic=[280, 8, 1])
    assert rc == -6 and "torque-driven" in msg


def test_factor_cache_checks():
    """The factor cache belongs to the persistent path of torque-driven models: any other path,
    a muscle model or a flag other than 0 / 1 is refused at sim_create."""
    ant = wl.workload("ant", 4)["model"]
    for kw, code, text in ((dict(factor_cache=2), -1, "factor_cache"),
                           (dict(factor_cache=1, path=2, k=1), -1, "persistent"),
                           (dict(factor_cache=1, path=1, k=1), -1, "persistent")):
        rc, msg = _create(ant, **kw)
        assert rc == code and text in msg, (kw, rc, msg)
    rc, msg = _create(wl.mtu_humanoid(), factor_cache=1, critic=[280, 8, 1])
    assert rc == -6 and "torque-driven" in msg


def test_layer_norm_checks():
    """layer_norm takes 0 or 1 and runs with FP32 / FP64 networks, not the BF16 matrix-core
    MLPs."""
    ant = wl.workload("ant", 4)["model"]
    rc, msg = _create(ant, layer_norm=2)
    assert rc == -1 and "layer_norm" in msg
    rc, msg = _create(ant, layer_norm=1, mlp_precision=1)
    assert rc == -6 and "layer normalisation" in msg
    rc, msg = _create(ant, layer_norm=1)
    assert rc in (0, -3), msg   # past the option checks (no device here: the first HIP call fails)
