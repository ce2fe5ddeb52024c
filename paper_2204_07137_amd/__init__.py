"""Python binding of libshacsim (argument marshalling only).

Every step of the window runs in the HIP kernels of ``libshacsim.so``; PyTorch is used
for device memory and streams.  Importing this package does not load the library;
``lib()`` does, and raises if the library is missing (there is no fallback).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# another build of the library (libshacsim_<name>.so, e.g. the phase-profiling build
# libshacsim_phase.so) is selected with SHACSIM_LIB=<name>
LIB_PATH = os.path.join(HERE, f"libshacsim_{os.environ['SHACSIM_LIB']}.so" if os.environ.get("SHACSIM_LIB")
                        else "libshacsim.so")

MAXL = 4
PATH_PERSISTENT, PATH_PLAIN, PATH_TAPE = 0, 1, 2
PREC = {"fp32": 0, "fp64": 1}
TASKS = {"none": 0, "cartpole": 1, "ant": 2, "humanoid": 3, "mtu": 4}
STATUS = {0: "SIM_OK", -1: "SIM_E_ARG", -2: "SIM_E_HANDLE", -3: "SIM_E_HIP", -4: "SIM_E_MODEL",
          -5: "SIM_E_WORKSPACE", -6: "SIM_E_UNSUPPORTED"}

_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_f = ctypes.c_float


class SimModelDesc(ctypes.Structure):
    _fields_ = [("n_joints", _i), ("parent", _p), ("jtype", _p), ("offset", _p), ("axis", _p),
                ("mass", _p), ("com", _p), ("inertia", _p), ("limited", _p), ("lower", _p),
                ("upper", _p), ("n_act", _i), ("act_joint", _p), ("gear", _p), ("armature", _p),
                ("n_contacts", _i), ("contact_body", _p), ("contact_pos", _p),
                ("contact_radius", _p), ("gravity", _d), ("kn", _d), ("kd", _d), ("kt", _d),
                ("mu", _d), ("klim", _d), ("dt", _d), ("substeps", _i), ("task", _i),
                ("has_last_action", _i), ("n_mtu", _i), ("mtu_npt", _p), ("mtu_body", _p),
                ("mtu_pos", _p), ("mtu_fmax", _p), ("mtu_lopt", _p), ("mtu_lslack", _p),
                ("tau_act", _d), ("fl_width", _d), ("vmax", _d), ("term_enabled", _i), ("term_height", _d)]


class SimOptions(ctypes.Structure):
    _fields_ = [("n_envs", _i), ("horizon", _i), ("ckpt_interval", _i), ("path", _i),
                ("closed_loop", _i), ("actor_layers", _i), ("actor_dims", _i * (MAXL + 1)),
                ("critic_layers", _i), ("critic_dims", _i * (MAXL + 1)), ("gamma", _d),
                ("precision", _i), ("chol_fp64_threshold", _d), ("policy_grad", _i),
                ("mlp_precision", _i), ("lanes_per_env", _i), ("factor_cache", _i), ("layer_norm", _i)]


class SimForwardIO(ctypes.Structure):
    _fields_ = [("s0", _p), ("actions_in", _p), ("actor_w", _p * MAXL), ("actor_b", _p * MAXL),
                ("critic_w", _p * MAXL), ("critic_b", _p * MAXL), ("actor_ln_g", _p * MAXL),
                ("actor_ln_b", _p * MAXL), ("critic_ln_g", _p * MAXL), ("critic_ln_b", _p * MAXL), ("workspace", _p),
                ("workspace_bytes", ctypes.c_size_t), ("s_h", _p), ("obs", _p), ("actions", _p),
                ("rewards", _p), ("value", _p), ("nonfinite", _p), ("fp64_refactor_count", _p),
                ("noise", _p), ("log_std", _p), ("reset_states", _p), ("done", _p),
                ("obs_mean", _p), ("obs_inv_std", _p), ("adhesive_count", _p), ("loss_env", _p), ("loss", _p)]


class SimAdjointIO(ctypes.Structure):
    _fields_ = [("s0", _p), ("actions", _p), ("obs", _p), ("s_h", _p),
                ("actor_w", _p * MAXL), ("actor_b", _p * MAXL), ("critic_w", _p * MAXL),
                ("critic_b", _p * MAXL), ("actor_ln_g", _p * MAXL), ("actor_ln_b", _p * MAXL),
                ("critic_ln_g", _p * MAXL), ("critic_ln_b", _p * MAXL), ("workspace", _p),
                ("workspace_bytes", ctypes.c_size_t), ("grad_s_h", _p), ("loss_scale", _d), ("dL_da", _p), ("dL_ds0", _p),
                ("dL_dtheta", _p), ("noise", _p), ("log_std", _p), ("dL_dlog_std", _p),
                ("obs_mean", _p), ("obs_inv_std", _p)]


class SimTuneResult(ctypes.Structure):
    _fields_ = [("path", _i), ("ckpt_interval", _i), ("workspace_bytes", ctypes.c_size_t),
                ("ms_window", _d), ("n_candidates", _i), ("lanes_per_env", _i), ("factor_cache", _i)]


class SimCriticFitIO(ctypes.Structure):
    _fields_ = [("obs", _p), ("targets", _p), ("rows", _i), ("perm", _p), ("n_iter", _i), ("n_minibatch", _i),
                ("critic_w", _p * MAXL), ("critic_b", _p * MAXL), ("adam_m", _p), ("adam_v", _p),
                ("adam_step", _i), ("lr", _d), ("beta1", _d), ("beta2", _d), ("eps", _d), ("loss_out", _p),
                ("workspace", _p), ("workspace_bytes", ctypes.c_size_t), ("obs_mean", _p), ("obs_inv_std", _p),
                ("critic_ln_g", _p * MAXL), ("critic_ln_b", _p * MAXL)]


EXPORTS = ["sim_create", "sim_workspace_bytes", "sim_dims", "sim_forward_window",
           "sim_adjoint_window", "sim_destroy", "sim_last_error", "sim_group_create",
           "sim_group_forward", "sim_group_adjoint", "sim_group_info", "sim_group_destroy",
           "sim_tune", "sim_probe_fma_bytes", "sim_probe_fma", "sim_probe_copy", "sim_adam_step",
           "sim_soft_update", "sim_td_lambda", "sim_critic_workspace_bytes", "sim_critic_values",
           "sim_critic_fit", "sim_obs_stats_update", "sim_abi_layout", "sim_critic_values_noalloc",
           "sim_critic_values_ln",
           "sim_phase_profile"]
MAX_GROUP = 6

_LIB = None


def lib():
    """Load libshacsim.so (built in-tree by build()).  Raises if it is absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2204_07137_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.sim_create.argtypes = [ctypes.POINTER(SimModelDesc), ctypes.POINTER(SimOptions), ctypes.POINTER(_p)]
        L.sim_create.restype = _i
        L.sim_workspace_bytes.argtypes = [_p]
        L.sim_workspace_bytes.restype = ctypes.c_size_t
        L.sim_dims.argtypes = [_p] + [ctypes.POINTER(_i)] * 5
        L.sim_dims.restype = _i
        L.sim_forward_window.argtypes = [_p, ctypes.POINTER(SimForwardIO), _p]
        L.sim_forward_window.restype = _i
        L.sim_adjoint_window.argtypes = [_p, ctypes.POINTER(SimAdjointIO), _p]
        L.sim_adjoint_window.restype = _i
        L.sim_destroy.argtypes = [_p]
        L.sim_destroy.restype = None
        L.sim_last_error.argtypes = []
        L.sim_last_error.restype = ctypes.c_char_p
        L.sim_group_create.argtypes = [ctypes.POINTER(_p), _i, ctypes.POINTER(_d), ctypes.POINTER(_p)]
        L.sim_group_create.restype = _i
        L.sim_group_forward.argtypes = [_p, ctypes.POINTER(SimForwardIO), _p]
        L.sim_group_forward.restype = _i
        L.sim_group_adjoint.argtypes = [_p, ctypes.POINTER(SimAdjointIO), _p]
        L.sim_group_adjoint.restype = _i
        L.sim_group_info.argtypes = [_p, ctypes.POINTER(_i), ctypes.POINTER(_i)]
        L.sim_group_info.restype = _i
        L.sim_group_destroy.argtypes = [_p]
        L.sim_group_destroy.restype = None
        L.sim_tune.argtypes = [ctypes.POINTER(SimModelDesc), ctypes.POINTER(SimOptions),
                               ctypes.POINTER(SimForwardIO), ctypes.c_size_t, _i, _p,
                               ctypes.POINTER(SimTuneResult)]
        L.sim_tune.restype = _i
        L.sim_probe_fma_bytes.argtypes = []
        L.sim_probe_fma_bytes.restype = ctypes.c_size_t
        L.sim_probe_fma.argtypes = [_p, ctypes.c_size_t, _p, ctypes.POINTER(_d)]
        L.sim_probe_fma.restype = _i
        L.sim_probe_copy.argtypes = [_p, _p, ctypes.c_size_t, _p, ctypes.POINTER(_d)]
        L.sim_probe_copy.restype = _i
        L.sim_adam_step.argtypes = [ctypes.POINTER(_p), ctypes.POINTER(ctypes.c_size_t), _i, _p, _p, _p, _i,
                                    _d, _d, _d, _d, _i, _p]
        L.sim_adam_step.restype = _i
        L.sim_soft_update.argtypes = [ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(ctypes.c_size_t), _i,
                                      _d, _i, _p]
        L.sim_soft_update.restype = _i
        L.sim_td_lambda.argtypes = [_p, _p, _p, _i, _i, _d, _d, _p, _i, _p]
        L.sim_td_lambda.restype = _i
        L.sim_critic_workspace_bytes.argtypes = [_p, _i]
        L.sim_critic_workspace_bytes.restype = ctypes.c_size_t
        L.sim_critic_values.argtypes = [_p, _p, _i, ctypes.POINTER(_p), ctypes.POINTER(_p), _p, _p, _p, _p,
                                        ctypes.c_size_t, _p]
        L.sim_critic_values.restype = _i
        L.sim_critic_values_ln.argtypes = [_p, _p, _i, ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p),
                                           ctypes.POINTER(_p), _p, _p, _p, _p, ctypes.c_size_t, _p]
        L.sim_critic_values_ln.restype = _i
        L.sim_critic_fit.argtypes = [_p, ctypes.POINTER(SimCriticFitIO), _p]
        L.sim_critic_fit.restype = _i
        L.sim_obs_stats_update.argtypes = [_p, ctypes.c_long, _i, _d, _p, _p, _p, _d, _i, _p]
        L.sim_obs_stats_update.restype = _i
        L.sim_critic_values_noalloc.argtypes = [_p, _p, _i, ctypes.POINTER(_p), ctypes.POINTER(_p), _p, _p, _p, _p]
        L.sim_critic_values_noalloc.restype = _i
        L.sim_abi_layout.argtypes = [_i, _i]
        L.sim_abi_layout.restype = ctypes.c_size_t
        L.sim_phase_profile.argtypes = [_p, _i, _i]
        L.sim_phase_profile.restype = _i
        _LIB = L
    return _LIB


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise SimError(code, lib().sim_last_error().decode())


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x), dtype=dtype)


def model_desc(md):
    """Build a SimModelDesc (and keep its host arrays alive) from a workload model dict."""
    keep = {}

    def ptr(name, arr, dtype):
        a = _arr(arr, dtype)
        keep[name] = a
        return a.ctypes.data_as(_p)

    d = SimModelDesc()
    d.n_joints = int(md["n_joints"])
    d.parent = ptr("parent", md["parent"], np.int32)
    d.jtype = ptr("jtype", md["jtype"], np.int32)
    d.offset = ptr("offset", md["offset"], np.float64)
    d.axis = ptr("axis", md["axis"], np.float64)
    d.mass = ptr("mass", md["mass"], np.float64)
    d.com = ptr("com", md["com"], np.float64)
    d.inertia = ptr("inertia", md["inertia"], np.float64)
    d.limited = ptr("limited", md["limited"], np.int32)
    d.lower = ptr("lower", md["lower"], np.float64)
    d.upper = ptr("upper", md["upper"], np.float64)
    d.n_act = int(md.get("n_motor", md["na"]))
    d.act_joint = ptr("act_joint", md["act_joint"], np.int32)
    d.gear = ptr("gear", md["gear"], np.float64)
    d.armature = ptr("armature", md["armature"], np.float64)
    d.n_contacts = int(len(md["contact_body"]))
    d.contact_body = ptr("contact_body", md["contact_body"], np.int32)
    d.contact_pos = ptr("contact_pos", np.reshape(md["contact_pos"], (-1, 3)), np.float64)
    d.contact_radius = ptr("contact_radius", md["contact_radius"], np.float64)
    for k in ("gravity", "kn", "kd", "kt", "mu", "klim", "dt"):
        setattr(d, k, float(md[k]))
    d.substeps = int(md["substeps"])
    d.task = TASKS[md["task"]]
    d.has_last_action = int(md["has_last_action"])
    d.n_mtu = int(md.get("n_mtu", 0))
    if d.n_mtu:
        d.mtu_npt = ptr("mtu_npt", md["mtu_npt"], np.int32)
        d.mtu_body = ptr("mtu_body", md["mtu_body"], np.int32)
        d.mtu_pos = ptr("mtu_pos", md["mtu_pos"], np.float64)
        d.mtu_fmax = ptr("mtu_fmax", md["mtu_fmax"], np.float64)
        d.mtu_lopt = ptr("mtu_lopt", md["mtu_lopt"], np.float64)
        d.mtu_lslack = ptr("mtu_lslack", md["mtu_lslack"], np.float64)
        d.tau_act = float(md["tau_act"])
        d.fl_width = float(md["fl_width"])
        d.vmax = float(md["vmax"])
    if md.get("term_height") is not None:
        d.term_enabled = 1
        d.term_height = float(md["term_height"])
    return d, keep


class Sim:
    """One handle: a model, a batch size N, a horizon h and the MLP shapes."""

    def __init__(self, md, n_envs, horizon, actor_dims=None, critic_dims=None, ckpt_interval=None,
                 path=PATH_PERSISTENT, gamma=0.99, precision="fp32", chol_fp64_threshold=1e-6,
                 policy_grad=False, mlp_precision="fp32", lanes_per_env=0, factor_cache=False, layer_norm=False):
        import torch
        self.torch = torch
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        L = lib()
        self.md = md
        d, self._keep = model_desc(md)
        self._desc = d
        o = SimOptions()
        o.n_envs = int(n_envs)
        o.horizon = int(horizon)
        o.ckpt_interval = int(ckpt_interval if ckpt_interval is not None else
                              (1 if path in (PATH_PLAIN, PATH_TAPE) else md["substeps"]))
        o.path = int(path)
        o.closed_loop = 1 if actor_dims is not None else 0
        if actor_dims is not None:
            o.actor_layers = len(actor_dims) - 1
            for i, v in enumerate(actor_dims):
                o.actor_dims[i] = int(v)
        o.critic_layers = len(critic_dims) - 1
        for i, v in enumerate(critic_dims):
            o.critic_dims[i] = int(v)
        o.gamma = float(gamma)
        o.precision = PREC[precision]
        o.chol_fp64_threshold = float(chol_fp64_threshold)
        o.policy_grad = 1 if policy_grad else 0
        o.mlp_precision = {"fp32": 0, "bf16": 1}[mlp_precision]
        o.lanes_per_env = int(lanes_per_env)
        o.factor_cache = 1 if factor_cache else 0
        o.layer_norm = 1 if layer_norm else 0
        self.layer_norm = bool(layer_norm)
        self.actor_dims = list(actor_dims) if actor_dims is not None else None
        h = _p()
        _check(L.sim_create(ctypes.byref(d), ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self.opt = o
        dims = [_i() for _ in range(5)]
        _check(L.sim_dims(h, *[ctypes.byref(x) for x in dims]))
        self.ns, self.od, self.na, self.nq, self.nv = (x.value for x in dims)
        self.N, self.H = int(n_envs), int(horizon)
        self.ws_bytes = int(L.sim_workspace_bytes(h))
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device="cuda")
        # serial number of the last forward enqueued on this handle's workspace: an adjoint
        # reads what its own forward left there, so it is refused once another forward ran
        self._fwd_serial = 0

    def _stamp(self, out):
        self._fwd_serial += 1
        out["_serial"] = self._fwd_serial

    def critic_workspace(self, rows):
        """A device workspace for critic_values / critic_fit on up to `rows` rows."""
        n = int(lib().sim_critic_workspace_bytes(self.h, int(rows)))
        return self.torch.empty(n, dtype=self.torch.uint8, device="cuda")

    def _norm_ptrs(self, obs_norm):
        if obs_norm is None:
            return _p(0), _p(0), None
        mean, inv_std = (self._dev(x).reshape(-1) for x in obs_norm)
        assert mean.shape == (self.od,) and inv_std.shape == (self.od,)
        return _p(mean.data_ptr()), _p(inv_std.data_ptr()), (mean, inv_std)

    def critic_values(self, obs, critic, workspace=None, obs_norm=None, critic_ln=None):
        """sim_critic_values: V(obs) for obs [rows, obs_dim] with critic [(W, b), ...] (device);
        obs_norm = (mean, inv_std) normalises the critic's input; critic_ln [(g, beta)] per hidden
        layer (a handle with layer_norm: sim_critic_values_ln)."""
        t = self.torch
        obs = self._dev(obs).reshape(-1, self.od)
        rows = obs.shape[0]
        ws = workspace if workspace is not None else self.critic_workspace(rows)
        cw = self.weights(critic)
        w = (_p * MAXL)(*([_p(W.data_ptr()) for W, _ in cw] + [_p(0)] * (MAXL - len(cw))))
        b = (_p * MAXL)(*([_p(B.data_ptr()) for _, B in cw] + [_p(0)] * (MAXL - len(cw))))
        out = t.empty(rows, device="cuda", dtype=self.dtype)
        pm, ps, keep = self._norm_ptrs(obs_norm)
        if critic_ln is None:
            _check(lib().sim_critic_values(self.h, _p(obs.data_ptr()), rows, w, b, pm, ps, _p(out.data_ptr()),
                                           _p(ws.data_ptr()), ws.numel(), _stream()))
        else:
            cln = [(self._dev(g).reshape(-1), self._dev(be).reshape(-1)) for g, be in critic_ln]
            lg = (_p * MAXL)(*([_p(g.data_ptr()) for g, _ in cln] + [_p(0)] * (MAXL - len(cln))))
            lb = (_p * MAXL)(*([_p(be.data_ptr()) for _, be in cln] + [_p(0)] * (MAXL - len(cln))))
            _check(lib().sim_critic_values_ln(self.h, _p(obs.data_ptr()), rows, w, b, lg, lb, pm, ps,
                                              _p(out.data_ptr()), _p(ws.data_ptr()), ws.numel(), _stream()))
            del cln
        del keep
        return out

    def critic_fit(self, obs, targets, perm, n_minibatch, critic, adam_m, adam_v, adam_step, lr,
                   beta1=0.7, beta2=0.95, eps=1e-8, workspace=None, obs_norm=None, critic_ln=None):
        """sim_critic_fit: fits `critic` (a list of device (W, b) tensors of this handle's dtype,
        updated in place) to targets [rows] on obs [rows, obs_dim] over len(perm) passes of
        n_minibatch minibatches (perm [n_iter, rows] int32).  With layer_norm, critic_ln is a
        list of device (g, beta) tensors per hidden layer, updated in place too, and the flat
        Adam moments hold W_0, b_0, g_0, beta_0, W_1, ...  Returns the minibatch losses."""
        t = self.torch
        obs = self._dev(obs).reshape(-1, self.od)
        targets = self._dev(targets).reshape(-1)
        rows = obs.shape[0]
        perm = perm.to(device="cuda", dtype=t.int32).contiguous()
        n_iter = perm.shape[0]
        ws = workspace if workspace is not None else self.critic_workspace(rows)
        losses = t.empty(n_iter * n_minibatch, device="cuda", dtype=self.dtype)
        io = SimCriticFitIO()
        io.obs, io.targets, io.rows = _p(obs.data_ptr()), _p(targets.data_ptr()), rows
        io.perm, io.n_iter, io.n_minibatch = _p(perm.data_ptr()), n_iter, int(n_minibatch)
        for i, (W, B) in enumerate(critic):
            assert W.dtype == self.dtype and W.is_cuda and W.is_contiguous() and B.is_contiguous()
            io.critic_w[i] = W.data_ptr()
            io.critic_b[i] = B.data_ptr()
        for i, (g, be) in enumerate(critic_ln or []):
            assert g.dtype == self.dtype and g.is_cuda and g.is_contiguous() and be.is_contiguous()
            io.critic_ln_g[i] = g.data_ptr()
            io.critic_ln_b[i] = be.data_ptr()
        io.adam_m, io.adam_v, io.adam_step = _p(adam_m.data_ptr()), _p(adam_v.data_ptr()), int(adam_step)
        io.lr, io.beta1, io.beta2, io.eps = float(lr), float(beta1), float(beta2), float(eps)
        io.loss_out = _p(losses.data_ptr())
        io.workspace, io.workspace_bytes = _p(ws.data_ptr()), ws.numel()
        io.obs_mean, io.obs_inv_std, keep = self._norm_ptrs(obs_norm)
        _check(lib().sim_critic_fit(self.h, ctypes.byref(io), _stream()))
        del keep
        return losses

    def close(self):
        if getattr(self, "h", None):
            lib().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def _dev(self, x):
        t = self.torch
        if isinstance(x, t.Tensor):
            return x.to(device="cuda", dtype=self.dtype).contiguous()
        return t.as_tensor(np.asarray(x), dtype=self.dtype, device="cuda").contiguous()

    def weights(self, layers):
        """[(W [out,in], b [out])] -> device float32 tensors."""
        return [(self._dev(W), self._dev(b)) for (W, b) in layers]

    @staticmethod
    def _ptr(t):
        return _p(t.data_ptr()) if t is not None else _p(0)

    def forward(self, s0, actor=None, critic=None, actions_in=None, stream=None, noise=None, log_std=None,
                reset_states=None, obs_norm=None, actor_ln=None, critic_ln=None):
        """Run sim_forward_window.  Returns a dict of device tensors.  noise [h, N, na] and
        log_std [na] select the stochastic policy y = mu(o) + exp(log_std) * noise;
        reset_states [N, ns] are the restart states of a model with early termination (the
        result then holds done [h, N]); obs_norm = (mean, inv_std) [obs_dim] normalises the
        networks' inputs (the adjoint takes it from the result); actor_ln / critic_ln (handle
        with layer_norm) are per hidden layer the (gain, bias) of its normalisation."""
        out, io = self.forward_io(s0, actor, critic, actions_in, noise=noise, log_std=log_std,
                                  reset_states=reset_states, obs_norm=obs_norm, actor_ln=actor_ln,
                                  critic_ln=critic_ln)
        t = self.torch
        st = stream if stream is not None else t.cuda.current_stream()
        _check(lib().sim_forward_window(self.h, ctypes.byref(io), _p(st.cuda_stream)))
        self._stamp(out)
        return out

    def forward_io(self, s0, actor=None, critic=None, actions_in=None, out=None, noise=None, log_std=None,
                   reset_states=None, obs_norm=None, actor_ln=None, critic_ln=None):
        """Allocate the forward outputs (or reuse those of `out`, a previous result) and
        fill a SimForwardIO (no launch)."""
        t = self.torch
        N, H = self.N, self.H
        s0 = self._dev(s0)
        assert s0.shape == (N, self.ns), (s0.shape, (N, self.ns))
        dt = self.dtype
        keys = ("s_h", "obs", "actions", "rewards", "value", "nonfinite", "fp64_refactor_count", "adhesive_count",
                "loss_env", "loss")
        prev_done = None
        if out is not None:
            prev_done = out.get("done")
            out = {k: out[k] for k in keys}
            out["s0"] = s0
        else:
            out = dict(
                s0=s0,
                s_h=t.empty(N, self.ns, device="cuda", dtype=dt),
                obs=t.empty(H + 1, N, self.od, device="cuda", dtype=dt),
                actions=t.empty(H, N, self.na, device="cuda", dtype=dt),
                rewards=t.empty(H, N, device="cuda", dtype=dt),
                value=t.empty(N, device="cuda", dtype=dt),
                nonfinite=t.zeros(N, dtype=t.uint8, device="cuda"),
                fp64_refactor_count=t.zeros(N, dtype=t.int32, device="cuda"),
                adhesive_count=t.zeros(N, dtype=t.int32, device="cuda"),
                loss_env=t.empty(N, device="cuda", dtype=dt),
                loss=t.empty(1, device="cuda", dtype=dt),
            )
        io = SimForwardIO()
        io.s0 = self._ptr(s0)
        if actions_in is not None:
            actions_in = self._dev(actions_in)
            assert actions_in.shape == (H, N, self.na)
            out["actions_in"] = actions_in
            io.actions_in = self._ptr(actions_in)
        if reset_states is not None:
            reset_states = self._dev(reset_states)
            assert reset_states.shape == (N, self.ns)
            out["reset_states"] = reset_states
            io.reset_states = self._ptr(reset_states)
            out["done"] = prev_done if prev_done is not None else t.zeros(H, N, dtype=t.uint8, device="cuda")
            io.done = self._ptr(out["done"])
        if noise is not None:
            noise = self._dev(noise)
            log_std = self._dev(log_std)
            assert noise.shape == (H, N, self.na) and log_std.shape == (self.na,)
            out["noise"], out["log_std"] = noise, log_std
            io.noise, io.log_std = self._ptr(noise), self._ptr(log_std)
        if obs_norm is not None:
            io.obs_mean, io.obs_inv_std, out["obs_norm"] = self._norm_ptrs(obs_norm)
        self._set_weights(io, actor, critic, out)
        self._set_ln(io, actor_ln, critic_ln, out)
        io.workspace = self._ptr(self.workspace)
        io.workspace_bytes = self.workspace.numel()
        for k in ("s_h", "obs", "actions", "rewards", "value", "nonfinite", "fp64_refactor_count", "adhesive_count",
                  "loss_env", "loss"):
            setattr(io, k, self._ptr(out[k]))
        out["_io"] = io
        return out, io

    def _set_ln(self, io, actor_ln, critic_ln, keep):
        """The layer normalisations' gains and biases (handle with layer_norm): device copies in
        the handle's dtype kept in `keep`, pointers into io."""
        if actor_ln is not None:
            aln = [(self._dev(g).reshape(-1).contiguous(), self._dev(b).reshape(-1).contiguous()) for g, b in actor_ln]
            keep["actor_ln"] = aln
            for i, (g, b) in enumerate(aln):
                io.actor_ln_g[i], io.actor_ln_b[i] = g.data_ptr(), b.data_ptr()
        if critic_ln is not None:
            cln = [(self._dev(g).reshape(-1).contiguous(), self._dev(b).reshape(-1).contiguous()) for g, b in critic_ln]
            keep["critic_ln"] = cln
            for i, (g, b) in enumerate(cln):
                io.critic_ln_g[i], io.critic_ln_b[i] = g.data_ptr(), b.data_ptr()

    def _set_weights(self, io, actor, critic, keep):
        if actor is not None:
            aw = self.weights(actor)
            keep["actor"] = aw
            for i, (W, b) in enumerate(aw):
                io.actor_w[i] = W.data_ptr()
                io.actor_b[i] = b.data_ptr()
        cw = self.weights(critic)
        keep["critic"] = cw
        for i, (W, b) in enumerate(cw):
            io.critic_w[i] = W.data_ptr()
            io.critic_b[i] = b.data_ptr()

    def adjoint(self, fw, actor=None, critic=None, grad_s_h=None, loss_scale=None, stream=None,
                want_theta=False):
        """Run sim_adjoint_window after forward() on the same handle and stream.

        loss_scale defaults to 1/(N h), the gradient of the actor loss itself.  With
        want_theta (handle created with policy_grad=True) the result also holds
        dL_dtheta, a list of (dW [out, in], db [out]) views of one flat buffer."""
        out, io = self.adjoint_io(fw, actor, critic, grad_s_h, loss_scale, want_theta)
        t = self.torch
        st = stream if stream is not None else t.cuda.current_stream()
        _check(lib().sim_adjoint_window(self.h, ctypes.byref(io), _p(st.cuda_stream)))
        return out

    def adjoint_io(self, fw, actor=None, critic=None, grad_s_h=None, loss_scale=None, want_theta=False,
                   out=None):
        """Allocate the adjoint outputs (or reuse those of `out`) and fill a SimAdjointIO.
        Raises if fw is not the result of the last forward run on this handle (the workspace
        then holds another window's checkpoints and activations)."""
        if fw.get("_serial") != self._fwd_serial:
            raise RuntimeError("adjoint of a stale forward: another forward ran on this handle since "
                               "(its workspace holds that window); run the forward again first")
        t = self.torch
        N, H = self.N, self.H
        dt = self.dtype
        prev = out
        if prev is not None:
            out = dict(dL_da=prev["dL_da"], dL_ds0=prev["dL_ds0"])
        else:
            out = dict(dL_da=t.empty(H, N, self.na, device="cuda", dtype=dt),
                       dL_ds0=t.empty(N, self.ns, device="cuda", dtype=dt))
        io = SimAdjointIO()
        io.s0 = self._ptr(fw["s0"])
        io.actions = self._ptr(fw["actions"])
        io.obs = self._ptr(fw["obs"])
        io.s_h = self._ptr(fw["s_h"])
        self._set_weights(io, actor if actor is not None else fw.get("actor"),
                          critic if critic is not None else fw["critic"], out)
        self._set_ln(io, fw.get("actor_ln"), fw.get("critic_ln"), out)
        io.workspace = self._ptr(self.workspace)
        io.workspace_bytes = self.workspace.numel()
        if grad_s_h is not None:
            grad_s_h = self._dev(grad_s_h)
            out["grad_s_h"] = grad_s_h
            io.grad_s_h = self._ptr(grad_s_h)
        io.loss_scale = float(1.0 / (N * H) if loss_scale is None else loss_scale)
        io.dL_da = self._ptr(out["dL_da"])
        io.dL_ds0 = self._ptr(out["dL_ds0"])
        if "obs_norm" in fw:
            io.obs_mean, io.obs_inv_std = self._ptr(fw["obs_norm"][0]), self._ptr(fw["obs_norm"][1])
        if "noise" in fw:
            io.noise, io.log_std = self._ptr(fw["noise"]), self._ptr(fw["log_std"])
            if want_theta:
                g = (prev["dL_dlog_std"] if prev is not None and "dL_dlog_std" in prev
                     else t.empty(self.na, device="cuda", dtype=dt))
                out["dL_dlog_std"] = g
                io.dL_dlog_std = self._ptr(g)
        if want_theta:
            dims = self.actor_dims
            nl = len(dims) - 1
            lnw = 2 * sum(dims[1:-1]) if self.layer_norm else 0
            n = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(nl)) + lnw
            flat = (prev["dL_dtheta_flat"] if prev is not None and "dL_dtheta_flat" in prev
                    else t.empty(n, device="cuda", dtype=dt))
            out["dL_dtheta_flat"] = flat
            io.dL_dtheta = self._ptr(flat)
            views, lnv, off = [], [], 0
            for i in range(nl):
                nw = dims[i] * dims[i + 1]
                views.append((flat[off:off + nw].view(dims[i + 1], dims[i]),
                              flat[off + nw:off + nw + dims[i + 1]]))
                off += nw + dims[i + 1]
                if self.layer_norm and i < nl - 1:
                    w = dims[i + 1]
                    lnv.append((flat[off:off + w], flat[off + w:off + 2 * w]))
                    off += 2 * w
            out["dL_dtheta"] = views
            if self.layer_norm:
                out["dL_dln"] = lnv
        out["_io"] = io
        return out, io


class Group:
    """A mixed-morphology batch: the windows of several Sim handles in one graph-captured
    kernel launch (sim_group_*).  cost_hint: optional per-env costs for the dispatch order."""

    def __init__(self, sims, cost_hint=None):
        import torch
        self.torch = torch
        self.sims = list(sims)
        n = len(self.sims)
        arr = (_p * n)(*[s.h for s in self.sims])
        hint = (_d * n)(*cost_hint) if cost_hint is not None else None
        g = _p()
        _check(lib().sim_group_create(arr, n, hint, ctypes.byref(g)))
        self.g = g

    def order(self):
        o = (_i * len(self.sims))()
        _check(lib().sim_group_info(self.g, o, None))
        return list(o)

    def captures(self):
        c = _i()
        _check(lib().sim_group_info(self.g, None, ctypes.byref(c)))
        return c.value

    def close(self):
        if getattr(self, "g", None):
            lib().sim_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, args, stream=None):
        """args: per member (s0, actor, critic[, actions_in]), or a dict of Sim.forward's
        keywords (noise, log_std, reset_states ...).  Returns per-member dicts.  The output
        tensors are kept and reused by the next call, so repeated calls with the same inputs
        replay one captured graph (copy results out before calling again)."""
        outs, ios = [], []
        prev = getattr(self, "_fw", None) or [None] * len(self.sims)
        for sim, a, pv in zip(self.sims, args, prev):
            o, io = sim.forward_io(**a, out=pv) if isinstance(a, dict) else sim.forward_io(*a, out=pv)
            outs.append(o)
            ios.append(io)
        arr = (SimForwardIO * len(ios))(*ios)
        st = stream if stream is not None else self.torch.cuda.current_stream()
        _check(lib().sim_group_forward(self.g, arr, _p(st.cuda_stream)))
        for sim, o in zip(self.sims, outs):
            sim._stamp(o)
        self._fw = outs
        return outs

    def adjoint(self, fws, want_theta=False, stream=None):
        outs, ios = [], []
        prev = getattr(self, "_ad", None) or [None] * len(self.sims)
        for sim, fw, pv in zip(self.sims, fws, prev):
            o, io = sim.adjoint_io(fw, want_theta=want_theta, out=pv)
            outs.append(o)
            ios.append(io)
        arr = (SimAdjointIO * len(ios))(*ios)
        st = stream if stream is not None else self.torch.cuda.current_stream()
        _check(lib().sim_group_adjoint(self.g, arr, _p(st.cuda_stream)))
        self._ad = outs
        return outs


def tune(md, n_envs, horizon, actor_dims, critic_dims, s0, actor, critic, budget_bytes,
         reps=3, precision="fp32", gamma=0.99):
    """Run sim_tune: the fastest launch configuration (path, k, layout) of this model within a
    workspace budget.  Returns a dict with path, ckpt_interval, lanes_per_env, factor_cache,
    workspace_bytes, ms_window and n_candidates."""
    import torch
    probe = Sim(md, n_envs, horizon, actor_dims, critic_dims, ckpt_interval=md["substeps"],
                precision=precision, gamma=gamma)
    out, io = probe.forward_io(s0, actor, critic)
    r = SimTuneResult()
    st = torch.cuda.current_stream()
    _check(lib().sim_tune(ctypes.byref(probe._desc), ctypes.byref(probe.opt), ctypes.byref(io),
                          int(budget_bytes), int(reps),
                          _p(st.cuda_stream), ctypes.byref(r)))
    probe.close()
    return {"path": r.path, "ckpt_interval": r.ckpt_interval, "lanes_per_env": r.lanes_per_env,
            "factor_cache": r.factor_cache, "workspace_bytes": r.workspace_bytes, "ms_window": r.ms_window, "n_candidates": r.n_candidates,
            "keep": out}


def _prec(t):
    import torch
    return {torch.float32: PREC["fp32"], torch.float64: PREC["fp64"]}[t.dtype]


def _stream():
    import torch
    return _p(torch.cuda.current_stream().cuda_stream)


def adam_step(params, grad, m, v, step, lr, beta1=0.7, beta2=0.95, eps=1e-8):
    """sim_adam_step: one Adam step on a list of device tensors whose gradient and moments are
    the flat tensors grad, m, v (in list order); m and v are updated in place."""
    n = len(params)
    ptrs = (_p * n)(*[_p(t.data_ptr()) for t in params])
    sizes = (ctypes.c_size_t * n)(*[t.numel() for t in params])
    _check(lib().sim_adam_step(ptrs, sizes, n, _p(grad.data_ptr()), _p(m.data_ptr()), _p(v.data_ptr()), int(step),
                               float(lr), float(beta1), float(beta2), float(eps), _prec(grad), _stream()))


def soft_update(target, online, alpha):
    """sim_soft_update: target_i <- alpha target_i + (1 - alpha) online_i for lists of tensors."""
    n = len(target)
    tp = (_p * n)(*[_p(t.data_ptr()) for t in target])
    op = (_p * n)(*[_p(t.data_ptr()) for t in online])
    sizes = (ctypes.c_size_t * n)(*[t.numel() for t in target])
    _check(lib().sim_soft_update(tp, op, sizes, n, float(alpha), _prec(target[0]), _stream()))


def td_lambda(rewards, values, gamma=0.99, lam=0.95, done=None):
    """sim_td_lambda: TD-lambda estimates [h, N] from rewards [h, N] and values [h+1, N];
    done [h, N] uint8 (the forward window's termination flags) stops the returns."""
    import torch
    h, N = rewards.shape
    out = torch.empty_like(rewards)
    dp = None
    if done is not None:
        assert done.dtype == torch.uint8 and tuple(done.shape) == (h, N) and done.is_cuda
        dp = _p(done.data_ptr())
    _check(lib().sim_td_lambda(_p(rewards.data_ptr()), _p(values.data_ptr()), dp, h, N, float(gamma), float(lam),
                               _p(out.data_ptr()), _prec(rewards), _stream()))
    return out


def obs_stats_update(obs, count, mean, var, inv_std, eps=1e-5):
    """sim_obs_stats_update: merges obs [rows, dim] (device) into the running statistics
    (count, mean [dim], var [dim]) in place, writes inv_std = 1 / sqrt(var + eps), and
    returns the new count."""
    obs = obs.reshape(-1, mean.numel())
    assert obs.is_contiguous() and all(x.dtype == obs.dtype and x.is_cuda for x in (mean, var, inv_std))
    rows, dim = obs.shape
    _check(lib().sim_obs_stats_update(_p(obs.data_ptr()), rows, dim, float(count), _p(mean.data_ptr()),
                                      _p(var.data_ptr()), _p(inv_std.data_ptr()), float(eps), _prec(obs), _stream()))
    return count + rows


PHASES = ["frame_begin", "fk", "velocities", "contacts", "muscles", "newton_euler", "subtree_sums",
          "bias_crba_columns", "crba", "cholesky", "factor_lds", "solve", "integrate", "tape_store", "commit",
          "checkpoint", "adj_seed", "adj_integrator", "adj_lambda", "adj_path_sums", "adj_contacts",
          "adj_muscles", "adj_body_terms", "adj_subtree_sums", "adj_derivatives", "adj_state", "tape_load",
          "tape_prefetch", "adj_frame", "window_end", "termination", "fc_states", "muscle_paths",
          "muscle_accumulate", "adj_muscle_paths", "adj_muscle_derivatives", "adj_muscle_accumulate",
          "frame_obs", "frame_actor", "adj_frame_actor"]


def phase_profile(reset=True):
    """Per-phase shader-clock cycle totals of the window kernels since the last reset (a
    library built with --phase-profile and loaded with SHACSIM_LIB=phase), as {phase: cycles}."""
    L = lib()
    buf = (ctypes.c_ulonglong * 40)()
    n = L.sim_phase_profile(ctypes.cast(buf, _p), 40, 1 if reset else 0)
    if n < 0:
        _check(n)
    return {name: int(buf[i]) for i, name in enumerate(PHASES)}


def probe_ceilings(copy_bytes=1 << 30):
    """Measured device ceilings: FP32 VALU TFLOP/s of an FMA loop and GB/s (read + write)
    of a device copy of copy_bytes, both from the library's own probe kernels."""
    import torch
    st = torch.cuda.current_stream()
    L = lib()
    nb = int(L.sim_probe_fma_bytes())
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    tf = ctypes.c_double()
    _check(L.sim_probe_fma(_p(scratch.data_ptr()), nb, _p(st.cuda_stream), ctypes.byref(tf)))
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    gb = ctypes.c_double()
    _check(L.sim_probe_copy(_p(src.data_ptr()), _p(dst.data_ptr()), copy_bytes, _p(st.cuda_stream),
                            ctypes.byref(gb)))
    return {"fp32_valu_tflops": tf.value, "copy_gbs": gb.value, "copy_bytes": copy_bytes}


def window_function(noise=None, reset_states=None, obs_norm=None):
    """torch.autograd.Function over one window: forward -> sim_forward_window, backward ->
    sim_adjoint_window.

    ``ShacWindow.apply(sim, s0, actions_in, critic, *actor_params)`` with actor_params the
    flat sequence W_0, b_0, W_1, b_1, ... returns (loss, s_h, obs, actions, rewards,
    value).  Gradients flow to s0 (total, through the closed-loop policy), to actions_in
    in open loop, and to the actor parameters when the handle was created with
    policy_grad=True.  The loss is the short-horizon actor loss, as the forward window computes
    it (the loss output of sim_forward_window); a gradient
    arriving on s_h is propagated through the window as well.

    The returned class is bound to the optional inputs given here: noise [h, N, na] selects
    the stochastic policy, whose log_std [na] is then the LAST element of actor_params (and
    receives dL/dlog_std); reset_states [N, ns] enables early termination (the handle's
    model has a termination height); obs_norm = (mean, inv_std) normalises the networks'
    inputs."""
    import torch

    class ShacWindow(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim, s0, actions_in, critic, *actor_params):
            params = list(actor_params)
            log_std = params.pop().detach() if noise is not None else None
            actor = ([(params[2 * i].detach(), params[2 * i + 1].detach())
                      for i in range(len(params) // 2)] if params else None)
            fw = sim.forward(s0.detach(), actor, critic,
                             actions_in.detach() if actions_in is not None else None, noise=noise,
                             log_std=log_std, reset_states=reset_states, obs_norm=obs_norm)
            loss = fw["loss"].reshape(())
            ctx.sim, ctx.fw, ctx.open_loop = sim, fw, actions_in is not None
            ctx.n_actor = len(actor_params)
            ctx.mark_non_differentiable(fw["obs"], fw["actions"], fw["rewards"], fw["value"])
            return loss, fw["s_h"], fw["obs"], fw["actions"], fw["rewards"], fw["value"]

        @staticmethod
        def backward(ctx, g_loss, g_sh, *unused):
            sim, fw = ctx.sim, ctx.fw
            scale = float(g_loss) / (sim.N * sim.H) if g_loss is not None else 0.0
            want = bool(ctx.n_actor) and bool(sim.opt.policy_grad) and any(ctx.needs_input_grad[4:])
            ad = sim.adjoint(fw, grad_s_h=g_sh, loss_scale=scale, want_theta=want)
            gs0 = ad["dL_ds0"]
            ga = ad["dL_da"] if ctx.open_loop else None
            gth = [None] * ctx.n_actor
            if want:
                gth = [x for pair in ad["dL_dtheta"] for x in pair]
                if noise is not None:
                    gth.append(ad["dL_dlog_std"])
            return (None, gs0, ga, None, *gth)

    return ShacWindow
