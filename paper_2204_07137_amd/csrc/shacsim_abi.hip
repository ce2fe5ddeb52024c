// Host side of the C ABI: model validation and upload, workspace layout, argument
// checks and dispatch to the FP32 or FP64 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/shacsim.h"
#include "sim_types.h"

static_assert(SIM_MAX_JOINTS == SIM_MAXJ, "limit mismatch");
static_assert(SIM_MAX_DOFS == SIM_MAXV, "limit mismatch");
static_assert(SIM_MAX_CONTACTS == SIM_MAXC, "limit mismatch");
static_assert(SIM_MAX_ACTIONS == SIM_MAXA, "limit mismatch");
static_assert(SIM_MAX_HIDDEN == SIM_MAXHID, "limit mismatch");
static_assert(SIM_MAX_OBS == SIM_MAXOBS, "limit mismatch");
static_assert(SIM_MAX_LAYERS == SIM_MAXL, "limit mismatch");

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------- allocation-free critic values
// The scratch of sim_critic_values_noalloc (the critic's hidden-layer activations) is a
// static device array, held by every GPU the library runs on until the process ends.  In host
// code its name is only a host-side stand-in: the device address is taken once per device at
// set-up (sim_create, or the entry point's first call on a device) with hipGetSymbolAddress,
// and only that address is passed to kernels.
#define SIM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define SIM_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[SIM_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SIM_MAX_DEVICES];

// the device address of `scratch` on device dev, which must be the current device
static void* scratch_on_device(int dev) {
  if (dev < 0 || dev >= SIM_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------- phase profile
// A build with -DSIM_PHASE_PROFILE gives the window kernels this table of per-phase cycle
// totals (device address per device, as for the scratch above); sim_phase_profile reads it.
#ifdef SIM_PHASE_PROFILE
static __device__ unsigned long long phase_table[SIM_NPHASE];
static unsigned long long* g_phase_ptr[SIM_MAX_DEVICES];
static unsigned long long* phase_on_device(int dev) {
  if (dev < 0 || dev >= SIM_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_phase_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(phase_table)) != hipSuccess) return nullptr;
    g_phase_ptr[dev] = static_cast<unsigned long long*>(p);
  }
  return g_phase_ptr[dev];
}
#endif

static const uint32_t kMagic = 0x53484143u;

struct SimHandle {
  DevModelT<float> m32;
  DevModelT<double> m64;
  void* dev_model = nullptr;
  SimOptions opt;
  int ns = 0, od = 0, nq = 0, nv = 0, na = 0, substeps = 0;
  size_t elem = 4;
  size_t wt_actor_off[SIM_MAXL], wt_critic_off[SIM_MAXL], wp_actor_off[SIM_MAXL], wp_critic_off[SIM_MAXL];
  size_t bf_actor_off[SIM_MAXL][2], bf_critic_off[SIM_MAXL][2];   // BF16 forward / adjoint tiles
  size_t off_ckpt = 0, off_adj = 0, off_tape = 0, off_done = 0, off_seg = 0, off_hid = 0, ws_bytes = 0;
  int hid_w = 0;   // the actor's hidden widths, summed (closed loop)
  int tape_ws = 0;   // reals between consecutive tape entries
  int fc_ws = 0;     // reals between consecutive factor-cache entries
  size_t off_th_y = 0, off_th_lnp = 0;   // policy gradient with layer normalisation
  size_t off_fc = 0, off_fcq = 0;
  // policy-gradient scratch: two layer-adjoint buffers, split partials (the hidden
  // activations are the window's own, at off_hid)
  size_t off_th_d0 = 0, off_th_d1 = 0, off_th_part = 0;
  int th_splits = 0;
  int n_ckpt = 0;
  int device = -1;
  uint32_t magic = kMagic;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- ABI layout
// Byte offsets of the members of the ABI structures, in declaration order, as compiled here.
static const size_t kLayoutSimModelDesc[] = {
    offsetof(SimModelDesc, n_joints), offsetof(SimModelDesc, parent), offsetof(SimModelDesc, jtype),
    offsetof(SimModelDesc, offset), offsetof(SimModelDesc, axis), offsetof(SimModelDesc, mass),
    offsetof(SimModelDesc, com), offsetof(SimModelDesc, inertia), offsetof(SimModelDesc, limited),
    offsetof(SimModelDesc, lower), offsetof(SimModelDesc, upper), offsetof(SimModelDesc, n_act),
    offsetof(SimModelDesc, act_joint), offsetof(SimModelDesc, gear), offsetof(SimModelDesc, armature),
    offsetof(SimModelDesc, n_contacts), offsetof(SimModelDesc, contact_body),
    offsetof(SimModelDesc, contact_pos), offsetof(SimModelDesc, contact_radius),
    offsetof(SimModelDesc, gravity), offsetof(SimModelDesc, kn), offsetof(SimModelDesc, kd),
    offsetof(SimModelDesc, kt), offsetof(SimModelDesc, mu), offsetof(SimModelDesc, klim),
    offsetof(SimModelDesc, dt), offsetof(SimModelDesc, substeps), offsetof(SimModelDesc, task),
    offsetof(SimModelDesc, has_last_action), offsetof(SimModelDesc, n_mtu), offsetof(SimModelDesc, mtu_npt),
    offsetof(SimModelDesc, mtu_body), offsetof(SimModelDesc, mtu_pos), offsetof(SimModelDesc, mtu_fmax),
    offsetof(SimModelDesc, mtu_lopt), offsetof(SimModelDesc, mtu_lslack), offsetof(SimModelDesc, tau_act),
    offsetof(SimModelDesc, fl_width), offsetof(SimModelDesc, vmax), offsetof(SimModelDesc, term_enabled),
    offsetof(SimModelDesc, term_height),
};
static const size_t kLayoutSimOptions[] = {
    offsetof(SimOptions, n_envs), offsetof(SimOptions, horizon), offsetof(SimOptions, ckpt_interval),
    offsetof(SimOptions, path), offsetof(SimOptions, closed_loop), offsetof(SimOptions, actor_layers),
    offsetof(SimOptions, actor_dims), offsetof(SimOptions, critic_layers), offsetof(SimOptions, critic_dims),
    offsetof(SimOptions, gamma), offsetof(SimOptions, precision), offsetof(SimOptions, chol_fp64_threshold),
    offsetof(SimOptions, policy_grad), offsetof(SimOptions, mlp_precision), offsetof(SimOptions, lanes_per_env),
    offsetof(SimOptions, factor_cache), offsetof(SimOptions, layer_norm),
};
static const size_t kLayoutSimForwardIO[] = {
    offsetof(SimForwardIO, s0), offsetof(SimForwardIO, actions_in), offsetof(SimForwardIO, actor_w),
    offsetof(SimForwardIO, actor_b), offsetof(SimForwardIO, critic_w), offsetof(SimForwardIO, critic_b),
    offsetof(SimForwardIO, actor_ln_g), offsetof(SimForwardIO, actor_ln_b), offsetof(SimForwardIO, critic_ln_g),
    offsetof(SimForwardIO, critic_ln_b), offsetof(SimForwardIO, workspace), offsetof(SimForwardIO, workspace_bytes), offsetof(SimForwardIO, s_h),
    offsetof(SimForwardIO, obs), offsetof(SimForwardIO, actions), offsetof(SimForwardIO, rewards),
    offsetof(SimForwardIO, value), offsetof(SimForwardIO, nonfinite),
    offsetof(SimForwardIO, fp64_refactor_count), offsetof(SimForwardIO, noise),
    offsetof(SimForwardIO, log_std), offsetof(SimForwardIO, reset_states), offsetof(SimForwardIO, done),
    offsetof(SimForwardIO, obs_mean), offsetof(SimForwardIO, obs_inv_std),
    offsetof(SimForwardIO, adhesive_count), offsetof(SimForwardIO, loss_env), offsetof(SimForwardIO, loss),
};
static const size_t kLayoutSimAdjointIO[] = {
    offsetof(SimAdjointIO, s0), offsetof(SimAdjointIO, actions), offsetof(SimAdjointIO, obs),
    offsetof(SimAdjointIO, s_h), offsetof(SimAdjointIO, actor_w), offsetof(SimAdjointIO, actor_b),
    offsetof(SimAdjointIO, critic_w), offsetof(SimAdjointIO, critic_b), offsetof(SimAdjointIO, actor_ln_g),
    offsetof(SimAdjointIO, actor_ln_b), offsetof(SimAdjointIO, critic_ln_g), offsetof(SimAdjointIO, critic_ln_b),
    offsetof(SimAdjointIO, workspace),
    offsetof(SimAdjointIO, workspace_bytes), offsetof(SimAdjointIO, grad_s_h),
    offsetof(SimAdjointIO, loss_scale), offsetof(SimAdjointIO, dL_da), offsetof(SimAdjointIO, dL_ds0),
    offsetof(SimAdjointIO, dL_dtheta), offsetof(SimAdjointIO, noise), offsetof(SimAdjointIO, log_std),
    offsetof(SimAdjointIO, dL_dlog_std), offsetof(SimAdjointIO, obs_mean),
    offsetof(SimAdjointIO, obs_inv_std),
};
static const size_t kLayoutSimTuneResult[] = {
    offsetof(SimTuneResult, path), offsetof(SimTuneResult, ckpt_interval),
    offsetof(SimTuneResult, workspace_bytes), offsetof(SimTuneResult, ms_window),
    offsetof(SimTuneResult, n_candidates), offsetof(SimTuneResult, lanes_per_env),
    offsetof(SimTuneResult, factor_cache),
};
static const size_t kLayoutSimCriticFitIO[] = {
    offsetof(SimCriticFitIO, obs), offsetof(SimCriticFitIO, targets), offsetof(SimCriticFitIO, rows),
    offsetof(SimCriticFitIO, perm), offsetof(SimCriticFitIO, n_iter), offsetof(SimCriticFitIO, n_minibatch),
    offsetof(SimCriticFitIO, critic_w), offsetof(SimCriticFitIO, critic_b), offsetof(SimCriticFitIO, adam_m),
    offsetof(SimCriticFitIO, adam_v), offsetof(SimCriticFitIO, adam_step), offsetof(SimCriticFitIO, lr),
    offsetof(SimCriticFitIO, beta1), offsetof(SimCriticFitIO, beta2), offsetof(SimCriticFitIO, eps),
    offsetof(SimCriticFitIO, loss_out), offsetof(SimCriticFitIO, workspace),
    offsetof(SimCriticFitIO, workspace_bytes), offsetof(SimCriticFitIO, obs_mean),
    offsetof(SimCriticFitIO, obs_inv_std), offsetof(SimCriticFitIO, critic_ln_g), offsetof(SimCriticFitIO, critic_ln_b),
};

extern "C" size_t sim_abi_layout(int which, int field) {
  const size_t* tab = nullptr;
  size_t n = 0, size = 0;
#define SIM_LAYOUT_CASE(id, S) \
  case id: tab = kLayout##S; n = sizeof(kLayout##S) / sizeof(size_t); size = sizeof(S); break;
  switch (which) {
    SIM_LAYOUT_CASE(SIM_ABI_MODEL_DESC, SimModelDesc)
    SIM_LAYOUT_CASE(SIM_ABI_OPTIONS, SimOptions)
    SIM_LAYOUT_CASE(SIM_ABI_FORWARD_IO, SimForwardIO)
    SIM_LAYOUT_CASE(SIM_ABI_ADJOINT_IO, SimAdjointIO)
    SIM_LAYOUT_CASE(SIM_ABI_TUNE_RESULT, SimTuneResult)
    SIM_LAYOUT_CASE(SIM_ABI_CRITIC_FIT_IO, SimCriticFitIO)
    default: return (size_t)-1;
  }
#undef SIM_LAYOUT_CASE
  if (field < 0) return size;
  return (size_t)field < n ? tab[field] : (size_t)-1;
}

extern "C" const char* sim_last_error(void) { return g_err.c_str(); }

// the muscle tables in the packed form the kernels read (one vector load per point and unit)
template <typename T>
static void pack_mtu_tables(DevModelT<T>& d) {
  for (int k = 0; k < SIM_MAXMPT; ++k)
    for (int i = 0; i < SIM_MAXMTU; ++i) {
      T* pt = &d.mtu_pt[(k * SIM_MAXMTU + i) * 4];
      for (int c = 0; c < 3; ++c) pt[c] = d.mtu_pos[(k * 3 + c) * SIM_MAXMTU + i];
      pt[3] = (T)d.mtu_body[k * SIM_MAXMTU + i];
    }
  for (int i = 0; i < SIM_MAXMTU; ++i) {
    T* pr = &d.mtu_par[i * 4];
    pr[0] = d.mtu_fmax[i]; pr[1] = d.mtu_lopt[i]; pr[2] = d.mtu_lslack[i]; pr[3] = (T)d.mtu_npt[i];
  }
}

template <typename T>
static void convert_model(const DevModelT<double>& s, DevModelT<T>& d) {
  std::memcpy(&d, &s, offsetof(DevModelT<double>, dt_sub));   // leading ints
  d.dt_sub = (T)s.dt_sub; d.g = (T)s.g; d.kn = (T)s.kn; d.kd = (T)s.kd; d.kt = (T)s.kt; d.mu = (T)s.mu;
  d.klim = (T)s.klim;
  d.chol_thr = (T)s.chol_thr;
  for (int j = 0; j < SIM_MAXJ; ++j) {
    d.parent[j] = s.parent[j]; d.jtype[j] = s.jtype[j]; d.qadr[j] = s.qadr[j]; d.vadr[j] = s.vadr[j];
    d.depth[j] = s.depth[j]; d.first_child[j] = s.first_child[j]; d.next_sib[j] = s.next_sib[j];
    d.act_of_joint[j] = s.act_of_joint[j]; d.limited[j] = s.limited[j];
    d.mass[j] = (T)s.mass[j]; d.lower[j] = (T)s.lower[j]; d.upper[j] = (T)s.upper[j]; d.gear[j] = (T)s.gear[j];
    for (int k = 0; k < 3; ++k) {
      d.offset[3 * j + k] = (T)s.offset[3 * j + k];
      d.axis[3 * j + k] = (T)s.axis[3 * j + k];
      d.com[3 * j + k] = (T)s.com[3 * j + k];
    }
    for (int k = 0; k < 6; ++k) d.inertia[6 * j + k] = (T)s.inertia[6 * j + k];
  }
  for (int i = 0; i < SIM_MAXV; ++i) d.armature[i] = (T)s.armature[i];
  for (int j = 0; j < SIM_MAXJ; ++j) {
    d.cmask[j] = s.cmask[j];
  }
  for (int g = 0; g < 4; ++g)
    for (int t = 0; t < SIM_MAXTS; ++t) d.ts_edge[g][t] = s.ts_edge[g][t];
  d.ts_steps = s.ts_steps;
  d.npair = s.npair;
  for (int p = 0; p < SIM_MAXPAIR; ++p) d.pair[p] = s.pair[p];
  d.tape_nw = s.tape_nw;
  for (int w = 0; w < SIM_MAXTAPEW; ++w) d.tape_off[w] = s.tape_off[w];
  d.fc_nw = s.fc_nw;
  for (int w = 0; w < SIM_MAXFCW; ++w) d.fc_off[w] = s.fc_off[w];
  d.tau_act = (T)s.tau_act; d.fl_w = (T)s.fl_w; d.vmax = (T)s.vmax;
  d.term_h = (T)s.term_h;
  for (int i = 0; i < SIM_MAXMTU; ++i) {
    d.mtu_npt[i] = s.mtu_npt[i];
    d.mtu_fmax[i] = (T)s.mtu_fmax[i]; d.mtu_lopt[i] = (T)s.mtu_lopt[i]; d.mtu_lslack[i] = (T)s.mtu_lslack[i];
  }
  for (int i = 0; i < SIM_MAXMPT * SIM_MAXMTU; ++i) d.mtu_body[i] = s.mtu_body[i];
  for (int i = 0; i < SIM_MAXMPT * 3 * SIM_MAXMTU; ++i) d.mtu_pos[i] = (T)s.mtu_pos[i];
  pack_mtu_tables(d);
  for (int c = 0; c < SIM_MAXC; ++c) {
    d.cbody[c] = s.cbody[c];
    d.crad[c] = (T)s.crad[c];
    for (int k = 0; k < 3; ++k) d.cpos[3 * c + k] = (T)s.cpos[3 * c + k];
  }
}

static int obs_dim_for(const DevModelT<double>& m) {
  if (m.task == TASK_CARTPOLE) return 5;
  if (m.task == TASK_ANT || m.task == TASK_HUMANOID) return 13 + 2 * (m.nq - 7) + (m.has_last_action ? m.na : 0);
  if (m.task == TASK_MTU) return 128 + m.n_mtu;
  return m.ns;   // no task: the observation is the state
}

static int build_model(const SimModelDesc* md, DevModelT<double>& m) {
  std::memset(&m, 0, sizeof(m));
  int J = md->n_joints;
  if (J < 1 || J > SIM_MAXJ) return fail(SIM_E_MODEL, "n_joints out of range [1, 32]");
  if (!md->parent || !md->jtype || !md->offset || !md->axis || !md->mass || !md->com || !md->inertia ||
      !md->limited || !md->lower || !md->upper || !md->armature)
    return fail(SIM_E_ARG, "sim_create: null model array");
  for (int j = 0; j < SIM_MAXJ; ++j) {
    m.first_child[j] = -1; m.next_sib[j] = -1; m.act_of_joint[j] = -1; m.parent[j] = -1; m.depth[j] = -1;
  }
  int nq = 0, nv = 0, maxd = 0;
  for (int j = 0; j < J; ++j) {
    int p = md->parent[j], t = md->jtype[j];
    if (p >= j || p < -1) return fail(SIM_E_MODEL, "parents must precede children");
    if (t != J_FREE && t != J_HINGE && t != J_SLIDE) return fail(SIM_E_MODEL, "unknown joint type");
    if (t == J_FREE && (p != -1 || j != 0)) return fail(SIM_E_MODEL, "a FREE joint must be frame 0 with no parent");
    m.parent[j] = p;
    m.jtype[j] = t;
    m.qadr[j] = nq;
    m.vadr[j] = nv;
    nq += (t == J_FREE) ? 7 : 1;
    nv += (t == J_FREE) ? 6 : 1;
    m.depth[j] = (p < 0) ? 0 : m.depth[p] + 1;
    maxd = std::max(maxd, m.depth[j]);
    for (int k = 0; k < 3; ++k) {
      m.offset[3 * j + k] = md->offset[3 * j + k];
      m.axis[3 * j + k] = md->axis[3 * j + k];
      m.com[3 * j + k] = md->com[3 * j + k];
    }
    const double* I = md->inertia + 9 * j;
    m.inertia[6 * j + 0] = I[0];
    m.inertia[6 * j + 1] = I[4];
    m.inertia[6 * j + 2] = I[8];
    m.inertia[6 * j + 3] = I[1];
    m.inertia[6 * j + 4] = I[2];
    m.inertia[6 * j + 5] = I[5];
    if (!(md->mass[j] >= 0.0)) return fail(SIM_E_MODEL, "negative mass");
    m.mass[j] = md->mass[j];
    m.limited[j] = md->limited[j] ? 1 : 0;
    m.lower[j] = md->lower[j];
    m.upper[j] = md->upper[j];
  }
  if (nv > SIM_MAXV || nq > SIM_MAXQ) return fail(SIM_E_MODEL, "more than 32 velocity DOFs");
  for (int j = J - 1; j >= 1; --j) {
    int p = m.parent[j];
    if (p >= 0) {
      m.next_sib[j] = m.first_child[p];
      m.first_child[p] = j;
    }
  }
  if (md->n_act < 0 || md->n_act > SIM_MAXA) return fail(SIM_E_MODEL, "n_act out of range [0, 32]");
  if (md->n_act > 0 && (!md->act_joint || !md->gear)) return fail(SIM_E_ARG, "null actuator arrays");
  for (int i = 0; i < md->n_act; ++i) {
    int j = md->act_joint[i];
    if (j < 0 || j >= J || m.jtype[j] == J_FREE || m.act_of_joint[j] >= 0)
      return fail(SIM_E_MODEL, "actuator must drive a distinct hinge or slide joint");
    m.act_of_joint[j] = i;
    m.gear[j] = md->gear[i];
  }
  for (int i = 0; i < nv; ++i) m.armature[i] = md->armature[i];
  if (md->n_contacts < 0 || md->n_contacts > SIM_MAXC) return fail(SIM_E_MODEL, "n_contacts out of range [0, 32]");
  if (md->n_contacts > 0 && (!md->contact_body || !md->contact_pos || !md->contact_radius))
    return fail(SIM_E_ARG, "null contact arrays");
  for (int c = 0; c < md->n_contacts; ++c) {
    int b = md->contact_body[c];
    if (b < 0 || b >= J) return fail(SIM_E_MODEL, "contact body out of range");
    m.cbody[c] = b;
    m.cmask[b] |= 1u << c;
    for (int k = 0; k < 3; ++k) m.cpos[3 * c + k] = md->contact_pos[3 * c + k];
    m.crad[c] = md->contact_radius[c];
  }
  if (md->substeps < 1 || !(md->dt > 0)) return fail(SIM_E_MODEL, "substeps >= 1 and dt > 0 required");
  if (md->n_mtu < 0 || md->n_mtu > SIM_MAXMTU) return fail(SIM_E_MODEL, "n_mtu out of range [0, 160]");
  if (md->n_mtu > 0) {
    if (!md->mtu_npt || !md->mtu_body || !md->mtu_pos || !md->mtu_fmax || !md->mtu_lopt || !md->mtu_lslack)
      return fail(SIM_E_ARG, "null muscle arrays");
    if (!(md->tau_act > 0) || !(md->fl_width > 0) || !(md->vmax > 0))
      return fail(SIM_E_MODEL, "tau_act, fl_width and vmax must be > 0");
    if (md->n_act + md->n_mtu > SIM_MAXAM) return fail(SIM_E_MODEL, "n_act + n_mtu above 160");
    if (md->has_last_action) return fail(SIM_E_UNSUPPORTED, "muscle models carry activations, not the last action");
    for (int i = 0; i < md->n_mtu; ++i) {
      const int np = md->mtu_npt[i];
      if (np < 2 || np > SIM_MAXMPT) return fail(SIM_E_MODEL, "a muscle path has 2..6 points");
      if (!(md->mtu_fmax[i] >= 0) || !(md->mtu_lopt[i] > 0) || !(md->mtu_lslack[i] >= 0))
        return fail(SIM_E_MODEL, "muscle F_max >= 0, l_opt > 0, l_slack >= 0 required");
      m.mtu_npt[i] = np;
      m.mtu_fmax[i] = md->mtu_fmax[i]; m.mtu_lopt[i] = md->mtu_lopt[i]; m.mtu_lslack[i] = md->mtu_lslack[i];
      // slots past the last point repeat it, so the kernels load every slot unconditionally
      for (int k = 0; k < SIM_MAXMPT; ++k) {
        const int kk = k < np ? k : np - 1;
        int b = md->mtu_body[i * SIM_MAXMPT + kk];
        if (b < 0 || b >= J) return fail(SIM_E_MODEL, "muscle point body out of range");
        m.mtu_body[k * SIM_MAXMTU + i] = b;
        for (int c = 0; c < 3; ++c)
          m.mtu_pos[(k * 3 + c) * SIM_MAXMTU + i] = md->mtu_pos[(i * SIM_MAXMPT + kk) * 3 + c];
      }
    }
    m.tau_act = md->tau_act; m.fl_w = md->fl_width; m.vmax = md->vmax;
  }
  pack_mtu_tables(m);
  if (md->task == TASK_MTU && md->n_mtu < 1) return fail(SIM_E_MODEL, "the muscle task needs muscles");
  m.J = J; m.nq = nq; m.nv = nv; m.na = md->n_act + md->n_mtu; m.nc = md->n_contacts;
  m.n_mtu = md->n_mtu; m.n_motor = md->n_act; m.nck = nq + nv + md->n_mtu;
  m.term = md->term_enabled ? 1 : 0;
  m.term_h = md->term_height;
  if (m.term && m.jtype[0] != J_FREE) return fail(SIM_E_MODEL, "early termination needs a FREE root");
  m.task = md->task; m.floating = (m.jtype[0] == J_FREE) ? 1 : 0;
  m.has_last_action = md->has_last_action ? 1 : 0;
  m.substeps = md->substeps; m.max_depth = maxd;
  {
    // Schedule of the forward subtree sums over four lane groups: an edge j -> parent(j) is
    // ready once every edge into j is done; each step takes up to four ready edges with
    // distinct parents, deepest child first (the longest remaining chain to the root).
    std::vector<int> pending(J, 0), done(J, 0);
    for (int j = 1; j < J; ++j)
      if (m.parent[j] >= 0) pending[m.parent[j]]++;
    for (int g = 0; g < 4; ++g)
      for (int t = 0; t < SIM_MAXTS; ++t) m.ts_edge[g][t] = 0;
    int left = 0;
    for (int j = 1; j < J; ++j) left += (m.parent[j] >= 0) ? 1 : 0;
    int steps = 0;
    while (left > 0) {
      if (steps >= SIM_MAXTS) return fail(SIM_E_MODEL, "subtree-sum schedule exceeds SIM_MAXTS steps");
      std::vector<int> ready;
      for (int j = 1; j < J; ++j)
        if (m.parent[j] >= 0 && !done[j] && pending[j] == 0) ready.push_back(j);
      std::stable_sort(ready.begin(), ready.end(), [&](int a, int b) { return m.depth[a] > m.depth[b]; });
      std::vector<int> taken;
      for (int j : ready) {
        if ((int)taken.size() == 4) break;
        bool clash = false;
        for (int t : taken) clash = clash || (m.parent[t] == m.parent[j]);
        if (!clash) taken.push_back(j);
      }
      for (size_t g = 0; g < taken.size(); ++g) {
        const int j = taken[g];
        m.ts_edge[g][steps] = (unsigned short)(j | (m.parent[j] << 5) | (1 << 10));
        done[j] = 1;
        --left;
      }
      for (int j : taken) pending[m.parent[j]]--;
      ++steps;
    }
    m.ts_steps = steps;
  }
  m.dt_sub = md->dt / md->substeps;
  m.g = md->gravity; m.kn = md->kn; m.kd = md->kd; m.kt = md->kt; m.mu = md->mu; m.klim = md->klim;
  m.ns = nq + nv + (m.has_last_action ? m.na : 0) + m.n_mtu;
  if (m.task == TASK_ANT || m.task == TASK_HUMANOID) {
    if (!m.floating) return fail(SIM_E_MODEL, "locomotion tasks need a FREE root");
  } else if (m.task == TASK_MTU) {
    if (!m.floating) return fail(SIM_E_MODEL, "locomotion tasks need a FREE root");
    if (13 + 2 * (nq - 7) > 128) return fail(SIM_E_MODEL, "muscle task: skeleton observation wider than 128");
  } else if (m.task == TASK_CARTPOLE) {
    if (nq != 2 || nv != 2) return fail(SIM_E_MODEL, "cartpole task needs a 2-DOF model");
  } else if (m.task != TASK_NONE) {
    return fail(SIM_E_MODEL, "unknown task");
  }
  m.od = obs_dim_for(m);
  if (m.od > SIM_MAXOBS) return fail(SIM_E_MODEL, "observation wider than 288");
  m.npair = 0;
  for (int i = 0; i < J; ++i) {
    if (m.jtype[i] == J_FREE) continue;
    for (int k = i; k >= 0; k = m.parent[k]) {
      if (m.npair >= SIM_MAXPAIR) return fail(SIM_E_MODEL, "too many mass-matrix pairs");
      m.pair[m.npair++] = i | (k << 5) | (m.vadr[i] << 10) | (m.vadr[k] << 15) |
                          ((m.jtype[k] == J_FREE ? 1 : 0) << 20) | (1 << 21);
    }
  }
  return SIM_OK;
}

static int check_options(const SimOptions* opt, const DevModelT<double>& m) {
  if (opt->n_envs < 1 || opt->horizon < 1) return fail(SIM_E_ARG, "n_envs and horizon must be >= 1");
  if (opt->ckpt_interval < 1 || m.substeps % opt->ckpt_interval != 0)
    return fail(SIM_E_ARG, "ckpt_interval must divide the substep count");
  if (opt->path != SIM_PATH_PERSISTENT && opt->path != SIM_PATH_PLAIN && opt->path != SIM_PATH_TAPE)
    return fail(SIM_E_ARG, "unknown path");
  if (opt->path == SIM_PATH_PLAIN && opt->ckpt_interval != 1)
    return fail(SIM_E_ARG, "the plain path stores every substep: ckpt_interval must be 1");
  if (opt->path == SIM_PATH_TAPE && opt->ckpt_interval != 1)
    return fail(SIM_E_ARG, "the tape path stores every substep: ckpt_interval must be 1");
  if (opt->precision != SIM_PREC_FP32 && opt->precision != SIM_PREC_FP64) return fail(SIM_E_ARG, "unknown precision");
  if (opt->critic_layers < 1 || opt->critic_layers > SIM_MAXL) return fail(SIM_E_ARG, "critic_layers out of range");
  if (opt->critic_dims[0] != m.od || opt->critic_dims[opt->critic_layers] != 1)
    return fail(SIM_E_ARG, "critic dims must map obs_dim to 1");
  for (int l = 0; l <= opt->critic_layers; ++l)
    if (opt->critic_dims[l] < 1 || opt->critic_dims[l] > SIM_MAXHID) return fail(SIM_E_ARG, "critic width out of range");
  if (opt->closed_loop) {
    if (opt->actor_layers < 1 || opt->actor_layers > SIM_MAXL) return fail(SIM_E_ARG, "actor_layers out of range");
    if (opt->actor_dims[0] != m.od || opt->actor_dims[opt->actor_layers] != m.na)
      return fail(SIM_E_ARG, "actor dims must map obs_dim to n_act");
    for (int l = 0; l <= opt->actor_layers; ++l)
      if (opt->actor_dims[l] < 1 || opt->actor_dims[l] > SIM_MAXHID) return fail(SIM_E_ARG, "actor width out of range");
  }
  if (opt->critic_layers > 3 || (opt->closed_loop && opt->actor_layers > 3))
    return fail(SIM_E_UNSUPPORTED, "at most two hidden layers per MLP");
  if (opt->policy_grad != 0 && opt->policy_grad != 1) return fail(SIM_E_ARG, "policy_grad must be 0 or 1");
  if (opt->policy_grad && !opt->closed_loop) return fail(SIM_E_ARG, "policy_grad needs the closed-loop policy");
  if (m.n_mtu > 0 && opt->path == SIM_PATH_PLAIN)
    return fail(SIM_E_UNSUPPORTED, "muscle models run on the persistent and tape paths");
  if (m.term && opt->path == SIM_PATH_PLAIN)
    return fail(SIM_E_UNSUPPORTED, "early termination runs on the persistent and tape paths");
  if (opt->mlp_precision != SIM_MLP_FP32 && opt->mlp_precision != SIM_MLP_BF16)
    return fail(SIM_E_ARG, "unknown mlp_precision");
  if (opt->mlp_precision == SIM_MLP_BF16 && opt->precision != SIM_PREC_FP32)
    return fail(SIM_E_ARG, "BF16 MLPs run in the FP32 path");
  if (opt->mlp_precision == SIM_MLP_BF16 && opt->policy_grad)
    return fail(SIM_E_UNSUPPORTED, "the policy-parameter gradient runs with FP32 MLPs");
  if (opt->layer_norm != 0 && opt->layer_norm != 1) return fail(SIM_E_ARG, "layer_norm must be 0 or 1");
  if (opt->layer_norm && opt->mlp_precision != SIM_MLP_FP32)
    return fail(SIM_E_UNSUPPORTED, "layer normalisation runs with FP32 / FP64 MLPs");
  if (opt->factor_cache != 0 && opt->factor_cache != 1) return fail(SIM_E_ARG, "factor_cache must be 0 or 1");
  if (opt->factor_cache && opt->path != SIM_PATH_PERSISTENT)
    return fail(SIM_E_ARG, "the factor cache belongs to the persistent (checkpointed) path");
  if (opt->factor_cache && m.n_mtu > 0) return fail(SIM_E_UNSUPPORTED, "the factor cache is for torque-driven models");
  if (opt->factor_cache && opt->ckpt_interval > SIM_FC_MAXK)
    return fail(SIM_E_UNSUPPORTED, "the factor cache takes checkpoint intervals up to 16");
  if (opt->lanes_per_env != 0) {
    const int ln = opt->lanes_per_env;
    if (ln != 16 && ln != 32 && ln != 64) return fail(SIM_E_ARG, "lanes_per_env must be 0, 16, 32 or 64");
    if (opt->precision != SIM_PREC_FP32 || opt->mlp_precision != SIM_MLP_FP32)
      return fail(SIM_E_UNSUPPORTED, "the compact layout runs in the FP32 path with FP32 MLPs");
    if (m.n_mtu > 0) return fail(SIM_E_UNSUPPORTED, "the compact layout is for torque-driven models");
    if (opt->path == SIM_PATH_PLAIN) return fail(SIM_E_UNSUPPORTED, "the compact layout runs on the persistent and tape paths");
    if (m.J > SIM_CJ || m.nv > SIM_CV || m.nc > SIM_CC || m.na > SIM_CA || m.od > SIM_COBS || m.npair > SIM_CPAIR)
      return fail(SIM_E_UNSUPPORTED, "model beyond the compact layout (16 frames, DOFs, contacts and actions, "
                                     "64 observations, 64 mass-matrix pairs)");
    if (m.J > ln || m.nv > ln || m.nc > ln || m.nq > ln)
      return fail(SIM_E_UNSUPPORTED, "frames, DOFs, contacts and coordinates must not exceed lanes_per_env");
    const int wmax = std::min(SIM_CHID, 8 * ln);
    for (int l = 0; l <= opt->critic_layers; ++l)
      if (opt->critic_dims[l] > wmax) return fail(SIM_E_UNSUPPORTED, "critic width beyond the compact layout");
    if (opt->closed_loop)
      for (int l = 0; l <= opt->actor_layers; ++l)
        if (opt->actor_dims[l] > wmax) return fail(SIM_E_UNSUPPORTED, "actor width beyond the compact layout");
    if (opt->n_envs % (SIM_WAVE / ln) != 0) return fail(SIM_E_ARG, "n_envs must be a multiple of 64 / lanes_per_env");
  }
  return SIM_OK;
}

// The 16-byte chunks of a packed tape entry (those holding a field the adjoint reads, at the
// model's own sizes) and the block offset of each, for the LDS layout the handle runs in
// (capacities J, V, C) and its element size: q, qd, S / v / ab / Ib of the frames, the
// contacts' force / point / velocity / depth, qdd, the lower triangle of the Cholesky factor row
// by row, the reciprocal pivots, the fallback flag, and for muscle models the frame rotations
// and positions and the activations.  The fields are in increasing block order, so a chunk
// shared by two runs is listed once.
static void build_tape_map(DevModelT<double>& m, int J, int V, int C, int elem) {
  const SimTapeLayout T = sim_tape_layout(J, V, C);
  const int wpc = 16 / elem;   // words per chunk
  int w = 0, last = -1;
  auto run = [&](int base, int n) {
    if (n <= 0) return;
    for (int c = base / wpc; c <= (base + n - 1) / wpc; ++c)
      if (c != last) { m.tape_off[w++] = (unsigned short)c; last = c; }
  };
  run(T.q, m.nq);
  run(T.qd, m.nv);
  run(T.S, 6 * m.J);
  run(T.v, 6 * m.J);
  run(T.ab, 6 * m.J);
  run(T.Ib, 10 * m.J);
  run(T.cf, 3 * m.nc);
  run(T.cx, 3 * m.nc);
  run(T.cvel, 3 * m.nc);
  run(T.cdep, m.nc);
  run(T.qdd, m.nv);
  for (int r = 0; r < m.nv; ++r) run(T.M + r * (V + 1), r + 1);
  run(T.tdinv, m.nv);
  run(T.tfb, 1);
  if (m.n_mtu > 0) {
    run(T.R, 9 * m.J);
    run(T.p, 3 * m.J);
    run(T.act, m.n_mtu);
  }
  m.tape_nw = w;
  for (int i = w; i < SIM_MAXTAPEW; ++i) m.tape_off[i] = 0;
}

// The 16-byte chunks of a factor-cache entry: the lower triangle of the Cholesky factor row by
// row, the reciprocal pivots and the fallback flag (the accelerations travel in a row of their
// own).
static void build_fc_map(DevModelT<double>& m, int J, int V, int C, int elem) {
  const SimTapeLayout T = sim_tape_layout(J, V, C);
  const int wpc = 16 / elem;
  int w = 0, last = -1;
  auto run = [&](int base, int n) {
    if (n <= 0) return;
    for (int c = base / wpc; c <= (base + n - 1) / wpc; ++c)
      if (c != last) { m.fc_off[w++] = (unsigned short)c; last = c; }
  };
  for (int r = 0; r < m.nv; ++r) run(T.M + r * (V + 1), r + 1);
  run(T.tdinv, m.nv);
  run(T.tfb, 1);
  m.fc_nw = w;
  for (int i = w; i < SIM_MAXFCW; ++i) m.fc_off[i] = 0;
}

extern "C" int sim_create(const SimModelDesc* md, const SimOptions* opt, SimHandle** out) {
  if (!md || !opt || !out) return fail(SIM_E_ARG, "sim_create: null argument");
  *out = nullptr;
  DevModelT<double> m;
  int rc = build_model(md, m);
  if (rc) return rc;
  rc = check_options(opt, m);
  if (rc) return rc;
  SimHandle* h = new SimHandle();
  m.chol_thr = opt->chol_fp64_threshold;
  {
    const int elem = (opt->precision == SIM_PREC_FP64) ? 8 : 4;
    if (opt->lanes_per_env) {
      build_tape_map(m, SIM_CJ, SIM_CV, SIM_CC, elem);
      build_fc_map(m, SIM_CJ, SIM_CV, SIM_CC, elem);
    } else {
      build_tape_map(m, SIM_MAXJ, SIM_MAXV, SIM_MAXC, elem);
      build_fc_map(m, SIM_MAXJ, SIM_MAXV, SIM_MAXC, elem);
    }
    const int fcap = sim_fc_chunk_cap(opt->lanes_per_env ? SIM_CV : SIM_MAXV, elem);
    if (m.fc_nw > fcap || m.fc_nw > SIM_MAXFCW) {
      delete h;
      return fail(SIM_E_MODEL, "sim_create: factor-cache entry beyond the layout's chunk capacity");
    }
    // the kernels hold an entry's chunk offsets in registers sized for this bound
    const int cap = opt->lanes_per_env ? sim_tape_chunk_cap(SIM_CJ, SIM_CV, SIM_CC, 0, elem)
                                       : sim_tape_chunk_cap(SIM_MAXJ, SIM_MAXV, SIM_MAXC, m.n_mtu > 0 ? SIM_MAXMTU : 0, elem);
    if (m.tape_nw > cap || m.tape_nw > SIM_MAXTAPEW) {
      delete h;
      return fail(SIM_E_MODEL, "sim_create: linearisation tape entry beyond the layout's chunk capacity");
    }
  }
  h->m64 = m;
  convert_model(m, h->m32);
  h->opt = *opt;
  h->ns = m.ns; h->od = m.od; h->nq = m.nq; h->nv = m.nv; h->na = m.na; h->substeps = m.substeps;
  h->elem = (opt->precision == SIM_PREC_FP64) ? 8 : 4;
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return fail(SIM_E_HIP, "hipGetDevice failed"); }
  if (!scratch_on_device(h->device)) {
    delete h;
    return fail(SIM_E_HIP, "sim_create: hipGetSymbolAddress of the static scratch failed on this device");
  }
  size_t msz = (opt->precision == SIM_PREC_FP64) ? sizeof(DevModelT<double>) : sizeof(DevModelT<float>);
  const void* src = (opt->precision == SIM_PREC_FP64) ? (const void*)&h->m64 : (const void*)&h->m32;
  if (hipMalloc(&h->dev_model, msz) != hipSuccess) { delete h; return fail(SIM_E_HIP, "hipMalloc failed"); }
  if (hipMemcpy(h->dev_model, src, msz, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(h->dev_model); delete h; return fail(SIM_E_HIP, "hipMemcpy failed");
  }
  // workspace: transposed MLP weights, checkpoint arena, plain-path adjoint, linearisation tape,
  // policy-gradient scratch
  const size_t e = h->elem;
  size_t off = 0;
  for (int l = 0; l < SIM_MAXL; ++l) {
    h->wt_actor_off[l] = h->wt_critic_off[l] = h->wp_actor_off[l] = h->wp_critic_off[l] = 0;
    h->bf_actor_off[l][0] = h->bf_actor_off[l][1] = h->bf_critic_off[l][0] = h->bf_critic_off[l][1] = 0;
  }
  if (opt->mlp_precision == SIM_MLP_BF16) {
    for (int l = 0; l < (opt->closed_loop ? opt->actor_layers : 0); ++l) {
      int ni = opt->actor_dims[l], no = opt->actor_dims[l + 1];
      h->bf_actor_off[l][0] = off;
      off = align256(off + sim_bf16_tiles_bytes(no, ni));
      h->bf_actor_off[l][1] = off;
      off = align256(off + sim_bf16_tiles_bytes(ni, no));
    }
    for (int l = 0; l < opt->critic_layers; ++l) {
      int ni = opt->critic_dims[l], no = opt->critic_dims[l + 1];
      h->bf_critic_off[l][0] = off;
      off = align256(off + sim_bf16_tiles_bytes(no, ni));
      h->bf_critic_off[l][1] = off;
      off = align256(off + sim_bf16_tiles_bytes(ni, no));
    }
  }
  auto pad64 = [](int n) { return (size_t)((n + SIM_WAVE - 1) / SIM_WAVE * SIM_WAVE); };
  if (opt->closed_loop)
    for (int l = 0; l < opt->actor_layers; ++l) {
      int ni = opt->actor_dims[l], no = opt->actor_dims[l + 1];
      h->wt_actor_off[l] = off;
      off = align256(off + e * ni * pad64(no));
      h->wp_actor_off[l] = off;
      off = align256(off + e * no * pad64(ni));
    }
  for (int l = 0; l < opt->critic_layers; ++l) {
    int ni = opt->critic_dims[l], no = opt->critic_dims[l + 1];
    h->wt_critic_off[l] = off;
    off = align256(off + e * ni * pad64(no));
    h->wp_critic_off[l] = off;
    off = align256(off + e * no * pad64(ni));
  }
  const size_t N = opt->n_envs, nqv = m.nck;
  h->n_ckpt = (opt->path == SIM_PATH_TAPE) ? 0
              : (opt->path == SIM_PATH_PLAIN) ? opt->horizon * m.substeps + 1
                                             : opt->horizon * m.substeps / opt->ckpt_interval;
  h->off_ckpt = off;
  off = align256(off + e * (size_t)h->n_ckpt * N * nqv);
  h->off_adj = off;
  off = align256(off + e * N * (nqv + m.na));
  // linearisation tape: every substep of the window (tape path) or one recomputed
  // segment but its last substep per env (persistent path); with the factor cache, the
  // pre-substep states of one segment per env instead
  const size_t tape_entries = (opt->path == SIM_PATH_TAPE) ? (size_t)opt->horizon * m.substeps * N
                              : (opt->path == SIM_PATH_PERSISTENT && !opt->factor_cache)
                                  ? N * (size_t)(opt->ckpt_interval - 1) : 0;
  h->off_tape = off;
  // packed entries of 16-byte chunks, each entry rounded up to 256 bytes
  h->tape_ws = (m.tape_nw * 16 / (int)e + 256 / (int)e - 1) / (256 / (int)e) * (256 / (int)e);
  off = align256(off + tape_entries * (size_t)h->tape_ws * e);
  if (opt->factor_cache) off = align256(off + e * N * (size_t)opt->ckpt_interval * nqv);
  // factor cache: [h S][N] entries and [h S][N][nv] accelerations
  h->fc_ws = opt->factor_cache ? (m.fc_nw * 16 / (int)e + 256 / (int)e - 1) / (256 / (int)e) * (256 / (int)e) : 0;
  h->off_fc = off;
  const size_t fc_subs = opt->factor_cache ? (size_t)opt->horizon * m.substeps * N : 0;
  off = align256(off + e * fc_subs * (size_t)h->fc_ws);
  h->off_fcq = off;
  off = align256(off + e * fc_subs * (size_t)m.nv);
  h->off_done = off;
  off = align256(off + (size_t)opt->horizon * N);
  h->off_seg = off;
  off = align256(off + (size_t)(opt->horizon + 1) * N * sizeof(int));
  h->hid_w = 0;
  if (opt->closed_loop) {
    for (int l = 1; l < opt->actor_layers; ++l) h->hid_w += opt->actor_dims[l];
    // with layer normalisation each hidden layer's mean and inverse deviation follow
    if (opt->layer_norm && opt->actor_layers > 1) h->hid_w += 2 * (opt->actor_layers - 1);
  }
  h->off_hid = off;
  off = align256(off + e * (size_t)opt->horizon * N * h->hid_w);
  if (opt->policy_grad) {
    const size_t rows = N * (size_t)opt->horizon;
    size_t maxw = 0, maxpart = 0;
    for (int l = 0; l < opt->actor_layers; ++l) {
      maxw = std::max(maxw, (size_t)opt->actor_dims[l + 1]);
      maxpart = std::max(maxpart, (size_t)opt->actor_dims[l + 1] * (opt->actor_dims[l] + 1));
    }
    // row chunks of at least 512 rows, at most 64 of them
    h->th_splits = (int)std::min<size_t>(64, std::max<size_t>(1, rows / 512));
    h->off_th_d0 = off;
    off = align256(off + e * rows * maxw);
    h->off_th_d1 = off;
    off = align256(off + e * rows * maxw);
    h->off_th_part = off;
    off = align256(off + e * (size_t)h->th_splits * maxpart);
    if (opt->layer_norm) {
      // the normalised hidden layers of every row and the gain / bias partials
      size_t hw = 0;
      for (int l = 1; l < opt->actor_layers; ++l) hw += opt->actor_dims[l];
      h->off_th_y = off;
      off = align256(off + e * rows * hw);
      h->off_th_lnp = off;
      off = align256(off + e * (size_t)SIM_LN_BLOCKS * 2 * maxw);
    }
  }
  h->ws_bytes = off;
  *out = h;
  g_err.clear();
  return SIM_OK;
}

extern "C" size_t sim_workspace_bytes(const SimHandle* h) {
  if (!h || h->magic != kMagic) return 0;
  return h->ws_bytes;
}

extern "C" int sim_dims(const SimHandle* h, int* n_state, int* n_obs, int* n_act, int* nq, int* nv) {
  if (!h || h->magic != kMagic) return fail(SIM_E_HANDLE, "invalid handle");
  if (n_state) *n_state = h->ns;
  if (n_obs) *n_obs = h->od;
  if (n_act) *n_act = h->na;
  if (nq) *nq = h->nq;
  if (nv) *nv = h->nv;
  return SIM_OK;
}

extern "C" void sim_destroy(SimHandle* h) {
  if (!h || h->magic != kMagic) return;
  h->magic = 0;
  if (h->dev_model) hipFree(h->dev_model);
  delete h;
}

static int check_handle(SimHandle* h) {
  if (!h || h->magic != kMagic) return fail(SIM_E_HANDLE, "invalid handle");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_E_HIP, "hipGetDevice failed");
  if (dev != h->device) return fail(SIM_E_ARG, "handle was created on another device");
  return SIM_OK;
}

template <typename T>
static int fill_mlp(MlpArgsT<T>& P, int nl, const int* dims, const void* const* W, const void* const* b,
                    char* ws, const size_t* wt_off, const size_t* wp_off, const size_t (*bf_off)[2], int bf16,
                    const char* what, int ln = 0, const void* const* lng = nullptr, const void* const* lnb = nullptr) {
  P.nl = nl;
  P.bf16 = bf16;
  P.ln = ln;
  P.ln_eps = (T)1e-5;
  for (int l = 0; l < SIM_MAXL; ++l) { P.lng[l] = nullptr; P.lnb[l] = nullptr; }
  if (ln)
    for (int l = 0; l + 1 < nl; ++l) {
      if (!lng || !lnb || !lng[l] || !lnb[l])
        return fail(SIM_E_ARG, std::string(what) + ": layer_norm needs every hidden layer's gain and bias");
      P.lng[l] = static_cast<const T*>(lng[l]);
      P.lnb[l] = static_cast<const T*>(lnb[l]);
    }
  for (int l = 0; l < SIM_MAXL; ++l) {
    P.Pf[l] = (bf16 && l < nl) ? reinterpret_cast<const uint16_t*>(ws + bf_off[l][0]) : nullptr;
    P.Pb[l] = (bf16 && l < nl) ? reinterpret_cast<const uint16_t*>(ws + bf_off[l][1]) : nullptr;
  }
  for (int l = 0; l <= SIM_MAXL; ++l) P.dims[l] = (l <= nl) ? dims[l] : 0;
  for (int l = 0; l < SIM_MAXL; ++l) { P.W[l] = nullptr; P.WT[l] = nullptr; P.b[l] = nullptr; P.src[l] = nullptr; }
  for (int l = 0; l < nl; ++l) {
    if (!W[l] || !b[l]) return fail(SIM_E_ARG, std::string(what) + ": null weight or bias pointer");
    P.src[l] = static_cast<const T*>(W[l]);
    P.b[l] = static_cast<const T*>(b[l]);
    P.WT[l] = reinterpret_cast<const T*>(ws + wt_off[l]);
    P.W[l] = reinterpret_cast<const T*>(ws + wp_off[l]);
  }
  return SIM_OK;
}

template <typename T>
static int launch_transposes(const MlpArgsT<T>& P, void* s);
template <>
int launch_transposes<float>(const MlpArgsT<float>& P, void* s) {
  for (int l = 0; l < P.nl; ++l) {
    int bad = P.bf16 ? sim_f32::launch_prep_bf16(P.src[l], const_cast<uint16_t*>(P.Pf[l]), const_cast<uint16_t*>(P.Pb[l]),
                                                 P.dims[l + 1], P.dims[l], s)
                     : sim_f32::launch_prep_weights(P.src[l], const_cast<float*>(P.WT[l]), const_cast<float*>(P.W[l]),
                                                    P.dims[l + 1], P.dims[l], s);
    if (bad) return -1;
  }
  return 0;
}
template <>
int launch_transposes<double>(const MlpArgsT<double>& P, void* s) {
  for (int l = 0; l < P.nl; ++l)
    if (sim_f64::launch_prep_weights(P.src[l], const_cast<double*>(P.WT[l]), const_cast<double*>(P.W[l]),
                                     P.dims[l + 1], P.dims[l], s))
      return -1;
  return 0;
}

// ---------------------------------------------------------------- argument building
template <typename T>
static int build_forward_args(SimHandle* h, const SimForwardIO* io, WinArgsT<T>& A) {
  const SimOptions& o = h->opt;
  char* ws = static_cast<char*>(io->workspace);
  std::memset(&A, 0, sizeof(A));
  A.model = static_cast<const DevModelT<T>*>(h->dev_model);
  A.N = o.n_envs; A.h = o.horizon; A.k = o.ckpt_interval; A.closed_loop = o.closed_loop;
  A.gamma = (T)o.gamma;
  A.scale = (T)(1.0 / ((double)o.n_envs * o.horizon));
  A.s0 = static_cast<const T*>(io->s0);
  A.actions_in = static_cast<const T*>(io->actions_in);
  A.noise = static_cast<const T*>(io->noise);
  A.log_std = static_cast<const T*>(io->log_std);
  int rc;
  if (o.closed_loop) {
    rc = fill_mlp(A.actor, o.actor_layers, o.actor_dims, io->actor_w, io->actor_b, ws, h->wt_actor_off, h->wp_actor_off,
                  h->bf_actor_off, o.mlp_precision == SIM_MLP_BF16, "actor", o.layer_norm, io->actor_ln_g,
                  io->actor_ln_b);
    if (rc) return rc;
  }
  rc = fill_mlp(A.critic, o.critic_layers, o.critic_dims, io->critic_w, io->critic_b, ws, h->wt_critic_off,
                h->wp_critic_off, h->bf_critic_off, o.mlp_precision == SIM_MLP_BF16, "critic", o.layer_norm,
                io->critic_ln_g, io->critic_ln_b);
  if (rc) return rc;
  A.s_h = static_cast<T*>(io->s_h); A.obs = static_cast<T*>(io->obs); A.actions = static_cast<T*>(io->actions);
  A.rewards = static_cast<T*>(io->rewards); A.value = static_cast<T*>(io->value);
  A.nonfinite = io->nonfinite;
  A.fallback = io->fp64_refactor_count;
  A.adhesive = io->adhesive_count;
  A.loss_env = static_cast<T*>(io->loss_env);
  A.loss = static_cast<T*>(io->loss);
  A.ckpt = reinterpret_cast<T*>(ws + h->off_ckpt);
  A.adj = reinterpret_cast<T*>(ws + h->off_adj);
  A.tape = reinterpret_cast<T*>(ws + h->off_tape);
  A.tape_full = (h->opt.path == SIM_PATH_TAPE);
  A.tape_ws = h->tape_ws;
  if (h->opt.factor_cache) {
    A.fc = reinterpret_cast<T*>(ws + h->off_fc);
    A.fcq = reinterpret_cast<T*>(ws + h->off_fcq);
    A.fc_ws = h->fc_ws;
  }
#ifdef SIM_PHASE_PROFILE
  A.prof = phase_on_device(h->device);
#endif
  A.reset = static_cast<const T*>(io->reset_states);
  A.done_out = io->done;
  A.done_ws = reinterpret_cast<uint8_t*>(ws + h->off_done);
  A.seg_ws = reinterpret_cast<int*>(ws + h->off_seg);
  A.obs_mean = static_cast<const T*>(io->obs_mean);
  A.obs_inv_std = static_cast<const T*>(io->obs_inv_std);
  A.hid = reinterpret_cast<T*>(ws + h->off_hid);
  A.hid_w = h->hid_w;
  return SIM_OK;
}

template <typename T>
static int build_adjoint_args(SimHandle* h, const SimAdjointIO* io, WinArgsT<T>& A) {
  const SimOptions& o = h->opt;
  char* ws = static_cast<char*>(io->workspace);
  std::memset(&A, 0, sizeof(A));
  A.model = static_cast<const DevModelT<T>*>(h->dev_model);
  A.N = o.n_envs; A.h = o.horizon; A.k = o.ckpt_interval; A.closed_loop = o.closed_loop;
  A.gamma = (T)o.gamma;
  A.scale = (T)io->loss_scale;
  A.s0 = static_cast<const T*>(io->s0);
  int rc;
  if (o.closed_loop) {
    rc = fill_mlp(A.actor, o.actor_layers, o.actor_dims, io->actor_w, io->actor_b, ws, h->wt_actor_off, h->wp_actor_off,
                  h->bf_actor_off, o.mlp_precision == SIM_MLP_BF16, "actor", o.layer_norm, io->actor_ln_g,
                  io->actor_ln_b);
    if (rc) return rc;
  }
  rc = fill_mlp(A.critic, o.critic_layers, o.critic_dims, io->critic_w, io->critic_b, ws, h->wt_critic_off,
                h->wp_critic_off, h->bf_critic_off, o.mlp_precision == SIM_MLP_BF16, "critic", o.layer_norm,
                io->critic_ln_g, io->critic_ln_b);
  if (rc) return rc;
  A.ckpt = reinterpret_cast<T*>(ws + h->off_ckpt);
  A.adj = reinterpret_cast<T*>(ws + h->off_adj);
  A.tape = reinterpret_cast<T*>(ws + h->off_tape);
  A.tape_full = (o.path == SIM_PATH_TAPE);
  A.tape_ws = h->tape_ws;
  if (h->opt.factor_cache) {
    A.fc = reinterpret_cast<T*>(ws + h->off_fc);
    A.fcq = reinterpret_cast<T*>(ws + h->off_fcq);
    A.fc_ws = h->fc_ws;
  }
#ifdef SIM_PHASE_PROFILE
  A.prof = phase_on_device(h->device);
#endif
  A.done_ws = reinterpret_cast<uint8_t*>(ws + h->off_done);
  A.seg_ws = reinterpret_cast<int*>(ws + h->off_seg);
  A.obs_in = static_cast<const T*>(io->obs);
  A.actions_fw = static_cast<const T*>(io->actions);
  A.s_h_in = static_cast<const T*>(io->s_h);
  A.grad_s_h = static_cast<const T*>(io->grad_s_h);
  A.dL_da = static_cast<T*>(io->dL_da);
  A.dL_ds0 = static_cast<T*>(io->dL_ds0);
  A.obs_mean = static_cast<const T*>(io->obs_mean);
  A.obs_inv_std = static_cast<const T*>(io->obs_inv_std);
  A.hid = reinterpret_cast<T*>(ws + h->off_hid);
  A.hid_w = h->hid_w;
  return SIM_OK;
}

template <typename T>
static void build_theta_args(SimHandle* h, const SimAdjointIO* io, ThetaArgsT<T>& P) {
  const SimOptions& o = h->opt;
  char* ws = static_cast<char*>(io->workspace);
  std::memset(&P, 0, sizeof(P));
  P.M = o.n_envs * o.horizon;
  P.nl = o.actor_layers;
  for (int l = 0; l <= o.actor_layers; ++l) P.dims[l] = o.actor_dims[l];
  P.splits = h->th_splits;
  long off = 0;
  for (int l = 0; l < o.actor_layers; ++l) {
    P.W[l] = static_cast<const T*>(io->actor_w[l]);
    P.b[l] = static_cast<const T*>(io->actor_b[l]);
    P.off_w[l] = off;
    off += (long)o.actor_dims[l] * o.actor_dims[l + 1];
    P.off_b[l] = off;
    off += o.actor_dims[l + 1];
    if (o.layer_norm && l + 1 < o.actor_layers) {
      // the hidden layer's normalisation gain and bias follow its W, b
      P.lng[l] = static_cast<const T*>(io->actor_ln_g[l]);
      P.lnb[l] = static_cast<const T*>(io->actor_ln_b[l]);
      P.off_g[l] = off;
      off += o.actor_dims[l + 1];
      P.off_beta[l] = off;
      off += o.actor_dims[l + 1];
    }
  }
  P.x0 = static_cast<const T*>(io->obs);
  P.x_shift = static_cast<const T*>(io->obs_mean);
  P.x_scale = static_cast<const T*>(io->obs_inv_std);
  P.act = static_cast<const T*>(io->actions);
  P.da = static_cast<const T*>(io->dL_da);
  P.d0 = reinterpret_cast<T*>(ws + h->off_th_d0);
  P.d1 = reinterpret_cast<T*>(ws + h->off_th_d1);
  P.part = reinterpret_cast<T*>(ws + h->off_th_part);
  P.out = static_cast<T*>(io->dL_dtheta);
  // the gradient is taken at the activations the window itself computed (stored by the
  // forward), rows (t, env) as the observations' (handles with BF16 MLPs have no dL/dtheta,
  // and an actor without hidden layers has none to store)
  if (h->hid_w > 0) {
    T* hid = reinterpret_cast<T*>(ws + h->off_hid);
    long off_l = 0;
    for (int l = 1; l < o.actor_layers; ++l) {
      P.H[l] = hid + off_l;
      P.ldH[l] = h->hid_w;
      off_l += o.actor_dims[l];
    }
    P.hidden_given = 1;
    if (o.layer_norm && o.actor_layers > 1) {
      P.ln = 1;
      P.st = hid + off_l;
      P.ldst = h->hid_w;
      T* y = reinterpret_cast<T*>(ws + h->off_th_y);
      long yo = 0;
      for (int l = 1; l < o.actor_layers; ++l) {
        P.Y[l] = y + yo;
        yo += (long)P.M * o.actor_dims[l];
      }
      P.lnpart = reinterpret_cast<T*>(ws + h->off_th_lnp);
      P.ln_blocks = SIM_LN_BLOCKS;
    }
  }
  P.mtu = (h->m64.task == TASK_MTU) ? 1 : 0;
  P.noise = static_cast<const T*>(io->noise);
  P.log_std = static_cast<const T*>(io->log_std);
  P.out_log_std = static_cast<T*>(io->dL_dlog_std);
}

// ---------------------------------------------------------------- launches (FP32 / FP64)
static int do_prep(const WinArgsT<float>& A, void* s) {
  int bad = A.closed_loop ? launch_transposes(A.actor, s) : 0;
  return bad | launch_transposes(A.critic, s);
}
static int do_prep(const WinArgsT<double>& A, void* s) {
  int bad = A.closed_loop ? launch_transposes(A.actor, s) : 0;
  return bad | launch_transposes(A.critic, s);
}
static int do_window(const WinArgsT<float>& A, int adjoint, int plain, int S, int nv, int mtu, int lanes, void* s) {
  return adjoint ? sim_f32::launch_adjoint(A, plain, S, nv, mtu, lanes, s)
                 : sim_f32::launch_forward(A, plain, S, nv, mtu, lanes, s);
}
static int do_window(const WinArgsT<double>& A, int adjoint, int plain, int S, int nv, int mtu, int lanes, void* s) {
  return adjoint ? sim_f64::launch_adjoint(A, plain, S, nv, mtu, lanes, s)
                 : sim_f64::launch_forward(A, plain, S, nv, mtu, lanes, s);
}
static int do_theta(const ThetaArgsT<float>& P, void* s) { return sim_f32::launch_theta(P, s); }
static int do_theta(const ThetaArgsT<double>& P, void* s) { return sim_f64::launch_theta(P, s); }
static int group_has_mtu(const int* mtu, int n) {
  for (int i = 0; i < n; ++i)
    if (mtu[i]) return 1;
  return 0;
}
static int do_group(const GroupArgsT<float>& G, int adjoint, size_t lds, void* s) {
  return sim_f32::launch_group(G, adjoint, group_has_mtu(G.mtu, G.n), lds, s);
}
static int do_group(const GroupArgsT<double>& G, int adjoint, size_t lds, void* s) {
  return sim_f64::launch_group(G, adjoint, group_has_mtu(G.mtu, G.n), lds, s);
}

static int launch_failed() {
  return fail(SIM_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
}

template <typename T>
static int run_forward(SimHandle* h, const SimForwardIO* io, void* stream) {
  WinArgsT<T> A;
  int rc = build_forward_args<T>(h, io, A);
  if (rc) return rc;
  int bad = do_prep(A, stream);
  bad |= do_window(A, 0, h->opt.path == SIM_PATH_PLAIN, h->substeps, h->nv, h->m64.n_mtu > 0, h->opt.lanes_per_env,
                   stream);
  return bad ? launch_failed() : SIM_OK;
}

template <typename T>
static int run_adjoint(SimHandle* h, const SimAdjointIO* io, void* stream) {
  WinArgsT<T> A;
  int rc = build_adjoint_args<T>(h, io, A);
  if (rc) return rc;
  if (do_window(A, 1, h->opt.path == SIM_PATH_PLAIN, h->substeps, h->nv, h->m64.n_mtu > 0, h->opt.lanes_per_env,
                stream))
    return launch_failed();
  if (io->dL_dtheta) {
    ThetaArgsT<T> P;
    build_theta_args<T>(h, io, P);
    if (do_theta(P, stream)) return launch_failed();
  }
  return SIM_OK;
}

// ---------------------------------------------------------------- argument checks
static int check_forward_io(SimHandle* h, const SimForwardIO* io) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!io) return fail(SIM_E_ARG, "null io");
  const SimOptions& o = h->opt;
  if (!io->s0 || !io->s_h || !io->obs || !io->actions || !io->rewards || !io->value)
    return fail(SIM_E_ARG, "sim_forward_window: null input/output pointer");
  if (!o.closed_loop && !io->actions_in) return fail(SIM_E_ARG, "open loop needs actions_in");
  if ((io->noise != nullptr) != (io->log_std != nullptr))
    return fail(SIM_E_ARG, "the stochastic policy needs both noise and log_std");
  if (io->noise && !o.closed_loop) return fail(SIM_E_ARG, "noise needs the closed-loop policy");
  if (h->m64.term && !io->reset_states) return fail(SIM_E_ARG, "early termination needs reset_states");
  if ((io->obs_mean != nullptr) != (io->obs_inv_std != nullptr))
    return fail(SIM_E_ARG, "observation normalisation needs both obs_mean and obs_inv_std");
  if (!io->workspace || io->workspace_bytes < h->ws_bytes)
    return fail(SIM_E_WORKSPACE, "workspace missing or smaller than sim_workspace_bytes()");
  return SIM_OK;
}

static int check_adjoint_io(SimHandle* h, const SimAdjointIO* io) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!io) return fail(SIM_E_ARG, "null io");
  const SimOptions& o = h->opt;
  if (!io->s0 || !io->actions || !io->obs || !io->s_h || !io->dL_da || !io->dL_ds0)
    return fail(SIM_E_ARG, "sim_adjoint_window: null input/output pointer");
  if (io->dL_dtheta && !o.policy_grad)
    return fail(SIM_E_ARG, "dL_dtheta needs a handle created with policy_grad = 1");
  if (io->dL_dtheta) {
    for (int l = 0; l < o.actor_layers; ++l)
      if (!io->actor_w[l] || !io->actor_b[l]) return fail(SIM_E_ARG, "dL_dtheta needs the actor weights");
  }
  if ((io->noise != nullptr) != (io->log_std != nullptr))
    return fail(SIM_E_ARG, "the stochastic policy needs both noise and log_std");
  if (io->dL_dlog_std && (!io->dL_dtheta || !io->noise))
    return fail(SIM_E_ARG, "dL_dlog_std needs dL_dtheta and the forward's noise and log_std");
  if ((io->obs_mean != nullptr) != (io->obs_inv_std != nullptr))
    return fail(SIM_E_ARG, "observation normalisation needs both obs_mean and obs_inv_std");
  if (!io->workspace || io->workspace_bytes < h->ws_bytes)
    return fail(SIM_E_WORKSPACE, "workspace missing or smaller than sim_workspace_bytes()");
  return SIM_OK;
}

extern "C" int sim_forward_window(SimHandle* h, const SimForwardIO* io, void* hip_stream) {
  int rc = check_forward_io(h, io);
  if (rc) return rc;
  return (h->opt.precision == SIM_PREC_FP64) ? run_forward<double>(h, io, hip_stream)
                                             : run_forward<float>(h, io, hip_stream);
}

extern "C" int sim_adjoint_window(SimHandle* h, const SimAdjointIO* io, void* hip_stream) {
  int rc = check_adjoint_io(h, io);
  if (rc) return rc;
  return (h->opt.precision == SIM_PREC_FP64) ? run_adjoint<double>(h, io, hip_stream)
                                             : run_adjoint<float>(h, io, hip_stream);
}

// ---------------------------------------------------------------- mixed-morphology groups
static const uint32_t kGroupMagic = 0x47525053u;

struct SimGroup {
  int n = 0, precision = 0, device = -1;
  SimHandle* h[SIM_MAXGROUP];
  int order[SIM_MAXGROUP];            // member in each work-table slot, decreasing per-env cost
  double cost[SIM_MAXGROUP];
  hipStream_t cap = nullptr;          // capture stream (default priority)
  hipGraphExec_t exec[2] = {nullptr, nullptr};   // forward, adjoint
  std::string key[2];                 // launch arguments the graph was captured with
  int captures = 0;
  size_t lds = 0;                     // LDS bytes of a group block: the largest a member needs
  uint32_t magic = kGroupMagic;
};

// Per-env cost estimate of one window: substeps times a per-substep operation count
// (factorisation, tree passes, contacts) plus the policy MLP per frame.
// blocks (wavefronts) of a member: one env each in the full layouts, 64 / lanes in the compact one
static int member_blocks(const SimHandle* h) {
  return h->opt.lanes_per_env ? h->opt.n_envs / (SIM_WAVE / h->opt.lanes_per_env) : h->opt.n_envs;
}

static double member_cost(const SimHandle* h) {
  const double nv = h->nv, J = h->m64.J, nc = h->m64.nc;
  double mlp = 0;
  for (int l = 0; l < h->opt.actor_layers; ++l) mlp += (double)h->opt.actor_dims[l] * h->opt.actor_dims[l + 1];
  return h->opt.horizon * (h->substeps * (nv * nv * nv / 3.0 + 2.0 * nv * nv + 900.0 * J + 120.0 * nc) + 3.0 * mlp);
}

static int check_group(SimGroup* g) {
  if (!g || g->magic != kGroupMagic) return fail(SIM_E_HANDLE, "invalid group");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_E_HIP, "hipGetDevice failed");
  if (dev != g->device) return fail(SIM_E_ARG, "group was created on another device");
  return SIM_OK;
}

extern "C" int sim_group_create(SimHandle* const* members, int n, const double* cost_hint, SimGroup** out) {
  if (!members || !out) return fail(SIM_E_ARG, "sim_group_create: null argument");
  *out = nullptr;
  if (n < 1 || n > SIM_MAXGROUP) return fail(SIM_E_ARG, "a group holds 1 to SIM_MAX_GROUP models");
  for (int i = 0; i < n; ++i) {
    int rc = check_handle(members[i]);
    if (rc) return rc;
    if (members[i]->opt.path == SIM_PATH_PLAIN)
      return fail(SIM_E_UNSUPPORTED, "group members must use the persistent or tape path");
    if (members[i]->opt.precision != members[0]->opt.precision)
      return fail(SIM_E_ARG, "group members must share one precision");
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return fail(SIM_E_ARG, "a handle appears twice in the group");
  }
  SimGroup* g = new SimGroup();
  g->n = n;
  g->precision = members[0]->opt.precision;
  g->device = members[0]->device;
  for (int i = 0; i < n; ++i) {
    g->h[i] = members[i];
    g->cost[i] = (cost_hint && cost_hint[i] > 0) ? cost_hint[i] : member_cost(members[i]);
    g->order[i] = i;
  }
  std::stable_sort(g->order, g->order + n, [g](int a, int b) { return g->cost[a] > g->cost[b]; });
  for (int i = 0; i < n; ++i) {
    const int lanes = members[i]->opt.lanes_per_env, mtu = members[i]->m64.n_mtu > 0;
    const size_t b = (g->precision == SIM_PREC_FP64) ? sim_f64::group_lds_bytes(lanes, mtu)
                                                     : sim_f32::group_lds_bytes(lanes, mtu);
    g->lds = std::max(g->lds, b);
  }
  const int prep = (g->precision == SIM_PREC_FP64) ? sim_f64::prepare_group(g->lds) : sim_f32::prepare_group(g->lds);
  if (prep) {
    delete g;
    return fail(SIM_E_HIP, "sim_group_create: the group kernels cannot be given the members' LDS");
  }
  if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return fail(SIM_E_HIP, "hipStreamCreate failed");
  }
  *out = g;
  g_err.clear();
  return SIM_OK;
}

extern "C" void sim_group_destroy(SimGroup* g) {
  if (!g || g->magic != kGroupMagic) return;
  g->magic = 0;
  for (int i = 0; i < 2; ++i)
    if (g->exec[i]) hipGraphExecDestroy(g->exec[i]);
  if (g->cap) hipStreamDestroy(g->cap);
  delete g;
}

extern "C" int sim_group_info(const SimGroup* g, int* order, int* n_captures) {
  if (!g || g->magic != kGroupMagic) return fail(SIM_E_HANDLE, "invalid group");
  if (order)
    for (int i = 0; i < g->n; ++i) order[i] = g->order[i];
  if (n_captures) *n_captures = g->captures;
  return SIM_OK;
}

// Captures `enqueue` on the group's stream into a graph (once per distinct argument set)
// and launches it on the caller's stream.
template <typename F>
static int group_launch(SimGroup* g, int which, const std::string& key, void* stream, F&& enqueue) {
  if (!g->exec[which] || g->key[which] != key) {
    if (g->exec[which]) {
      hipGraphExecDestroy(g->exec[which]);
      g->exec[which] = nullptr;
    }
    if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(SIM_E_HIP, "hipStreamBeginCapture failed");
    int bad = enqueue(static_cast<void*>(g->cap));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    if (bad || e != hipSuccess || !graph) {
      if (graph) hipGraphDestroy(graph);
      return fail(SIM_E_HIP, "graph capture of the group launch failed");
    }
    e = hipGraphInstantiate(&g->exec[which], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g->exec[which] = nullptr;
      return fail(SIM_E_HIP, "hipGraphInstantiate failed");
    }
    g->key[which] = key;
    g->captures++;
  }
  if (hipGraphLaunch(g->exec[which], (hipStream_t)stream) != hipSuccess) return fail(SIM_E_HIP, "hipGraphLaunch failed");
  return SIM_OK;
}

template <typename T>
static int run_group_forward(SimGroup* g, const SimForwardIO* ios, void* stream) {
  GroupArgsT<T> G;
  std::memset(&G, 0, sizeof(G));
  G.n = g->n;
  int start = 0;
  for (int s = 0; s < g->n; ++s) {
    SimHandle* h = g->h[g->order[s]];
    int rc = build_forward_args<T>(h, &ios[g->order[s]], G.A[s]);
    if (rc) return rc;
    G.start[s] = start;
    G.nv[s] = h->nv;
    G.mtu[s] = h->m64.n_mtu > 0;
    G.lanes[s] = h->opt.lanes_per_env;
    start += member_blocks(h);
  }
  G.start[g->n] = start;
  std::string key(reinterpret_cast<const char*>(&G), sizeof(G));
  return group_launch(g, 0, key, stream, [&](void* cs) {
    int bad = 0;
    for (int s = 0; s < G.n; ++s) bad |= do_prep(G.A[s], cs);
    return bad | do_group(G, 0, g->lds, cs);
  });
}

template <typename T>
static int run_group_adjoint(SimGroup* g, const SimAdjointIO* ios, void* stream) {
  GroupArgsT<T> G;
  std::memset(&G, 0, sizeof(G));
  G.n = g->n;
  ThetaArgsT<T> P[SIM_MAXGROUP];
  int has_theta[SIM_MAXGROUP];
  int start = 0;
  std::string key;
  for (int s = 0; s < g->n; ++s) {
    const int mi = g->order[s];
    SimHandle* h = g->h[mi];
    int rc = build_adjoint_args<T>(h, &ios[mi], G.A[s]);
    if (rc) return rc;
    G.start[s] = start;
    G.nv[s] = h->nv;
    G.mtu[s] = h->m64.n_mtu > 0;
    G.lanes[s] = h->opt.lanes_per_env;
    start += member_blocks(h);
    has_theta[s] = ios[mi].dL_dtheta != nullptr;
    if (has_theta[s]) {
      build_theta_args<T>(h, &ios[mi], P[s]);
      key.append(reinterpret_cast<const char*>(&P[s]), sizeof(P[s]));
    }
  }
  G.start[g->n] = start;
  key.append(reinterpret_cast<const char*>(&G), sizeof(G));
  return group_launch(g, 1, key, stream, [&](void* cs) {
    int bad = do_group(G, 1, g->lds, cs);
    for (int s = 0; s < G.n; ++s)
      if (has_theta[s]) bad |= do_theta(P[s], cs);
    return bad;
  });
}

extern "C" int sim_group_forward(SimGroup* g, const SimForwardIO* ios, void* hip_stream) {
  int rc = check_group(g);
  if (rc) return rc;
  if (!ios) return fail(SIM_E_ARG, "null io array");
  for (int i = 0; i < g->n; ++i) {
    rc = check_forward_io(g->h[i], &ios[i]);
    if (rc) return rc;
  }
  return g->precision == SIM_PREC_FP64 ? run_group_forward<double>(g, ios, hip_stream)
                                       : run_group_forward<float>(g, ios, hip_stream);
}

extern "C" int sim_group_adjoint(SimGroup* g, const SimAdjointIO* ios, void* hip_stream) {
  int rc = check_group(g);
  if (rc) return rc;
  if (!ios) return fail(SIM_E_ARG, "null io array");
  for (int i = 0; i < g->n; ++i) {
    rc = check_adjoint_io(g->h[i], &ios[i]);
    if (rc) return rc;
  }
  return g->precision == SIM_PREC_FP64 ? run_group_adjoint<double>(g, ios, hip_stream)
                                       : run_group_adjoint<float>(g, ios, hip_stream);
}

// ---------------------------------------------------------------- autotuner
// Times forward + adjoint windows for every launch configuration of one model whose
// workspace fits the budget (the tape path, then every checkpoint interval k dividing S)
// and reports the fastest.  A set-up call: it allocates and frees its own workspaces.
extern "C" int sim_tune(const SimModelDesc* model, const SimOptions* opt, const SimForwardIO* io,
                        size_t workspace_budget, int reps, void* hip_stream, SimTuneResult* out) {
  if (!model || !opt || !io || !out) return fail(SIM_E_ARG, "sim_tune: null argument");
  if (reps < 1) return fail(SIM_E_ARG, "sim_tune: reps must be >= 1");
  std::memset(out, 0, sizeof(*out));
  hipStream_t st = (hipStream_t)hip_stream;
  struct Cand { int path, k, lanes, fc; };
  std::vector<Cand> cands;
  for (int lanes : {0, 64, 32, 16}) {
    if (lanes) {
      // the compact layout only where the model and batch allow it
      SimOptions o = *opt;
      o.lanes_per_env = lanes;
      o.path = SIM_PATH_TAPE;
      o.ckpt_interval = 1;
      o.factor_cache = 0;
      DevModelT<double> m;
      if (build_model(model, m) || check_options(&o, m)) continue;
    }
    cands.push_back({SIM_PATH_TAPE, 1, lanes, 0});
    for (int k = 1; k <= model->substeps; ++k)
      if (model->substeps % k == 0) {
        cands.push_back({SIM_PATH_PERSISTENT, k, lanes, 0});
        SimOptions o = *opt;
        o.lanes_per_env = lanes;
        o.path = SIM_PATH_PERSISTENT;
        o.ckpt_interval = k;
        o.factor_cache = 1;
        DevModelT<double> m;
        if (!build_model(model, m) && !check_options(&o, m)) cands.push_back({SIM_PATH_PERSISTENT, k, lanes, 1});
      }
  }
  double best = -1.0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(SIM_E_HIP, "hipEventCreate failed");
  int rc = SIM_OK;
  for (const Cand& c : cands) {
    SimOptions o = *opt;
    o.path = c.path;
    o.ckpt_interval = c.k;
    o.lanes_per_env = c.lanes;
    o.factor_cache = c.fc;
    SimHandle* h = nullptr;
    rc = sim_create(model, &o, &h);
    if (rc) break;
    const size_t ws = h->ws_bytes;
    if (ws > workspace_budget) {
      sim_destroy(h);
      continue;
    }
    const size_t e = h->elem;
    void *wsp = nullptr, *da = nullptr, *ds0 = nullptr;
    if (hipMalloc(&wsp, ws > 0 ? ws : 256) != hipSuccess ||
        hipMalloc(&da, e * (size_t)o.horizon * o.n_envs * std::max(h->na, 1)) != hipSuccess ||
        hipMalloc(&ds0, e * (size_t)o.n_envs * h->ns) != hipSuccess) {
      if (wsp) hipFree(wsp);
      if (da) hipFree(da);
      sim_destroy(h);
      rc = fail(SIM_E_HIP, "sim_tune: hipMalloc failed");
      break;
    }
    SimForwardIO fio = *io;
    fio.workspace = wsp;
    fio.workspace_bytes = ws;
    SimAdjointIO aio;
    std::memset(&aio, 0, sizeof(aio));
    aio.s0 = io->s0; aio.actions = io->actions; aio.obs = io->obs; aio.s_h = io->s_h;
    for (int l = 0; l < SIM_MAXL; ++l) {
      aio.actor_w[l] = io->actor_w[l]; aio.actor_b[l] = io->actor_b[l];
      aio.critic_w[l] = io->critic_w[l]; aio.critic_b[l] = io->critic_b[l];
    }
    aio.workspace = wsp;
    aio.workspace_bytes = ws;
    aio.loss_scale = 1.0 / ((double)o.n_envs * o.horizon);
    aio.dL_da = da;
    aio.dL_ds0 = ds0;
    std::vector<float> t;
    for (int r = 0; r <= reps && rc == SIM_OK; ++r) {   // the first window is a warm-up
      hipEventRecord(e0, st);
      rc = sim_forward_window(h, &fio, st);
      if (!rc) rc = sim_adjoint_window(h, &aio, st);
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) rc = fail(SIM_E_HIP, "sim_tune: window failed");
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) t.push_back(ms);
    }
    hipFree(wsp);
    hipFree(da);
    hipFree(ds0);
    sim_destroy(h);
    if (rc) break;
    std::sort(t.begin(), t.end());
    const double med = t[t.size() / 2];
    out->n_candidates++;
    if (best < 0 || med < best) {
      best = med;
      out->path = c.path;
      out->ckpt_interval = c.k;
      out->workspace_bytes = ws;
      out->ms_window = med;
      out->lanes_per_env = c.lanes;
      out->factor_cache = c.fc;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (best < 0) return fail(SIM_E_WORKSPACE, "sim_tune: no configuration fits the workspace budget");
  g_err.clear();
  return SIM_OK;
}

// ======================================================================= device ceilings
// FP32 FMA loop: eight independent dependency chains per lane, no packed instructions
// (the build disables them), enough waves to fill every SIMD several times over.
#define PROBE_FMA_BLOCKS 4096
#define PROBE_FMA_THREADS 256
#define PROBE_FMA_ITERS 2048
__global__ __launch_bounds__(PROBE_FMA_THREADS) void k_probe_fma(float* out, float m, float c) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = (float)(threadIdx.x + j) * 1e-3f;
  for (int i = 0; i < PROBE_FMA_ITERS; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = __builtin_fmaf(a[j], m, c);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  out[(size_t)blockIdx.x * PROBE_FMA_THREADS + threadIdx.x] = s;
}

// device-to-device copy, 16 bytes per lane and step, grid-stride
__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// time fn(stream) (already warmed up once) with events on the stream; ms of one call
template <class F>
static int probe_time(F fn, hipStream_t s, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(SIM_E_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return fail(SIM_E_HIP, "hipEventCreate failed"); }
  fn();
  hipEventRecord(e0, s);
  fn();
  hipEventRecord(e1, s);
  const hipError_t err = hipEventSynchronize(e1);
  hipEventElapsedTime(ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess || hipGetLastError() != hipSuccess) return fail(SIM_E_HIP, "probe launch failed");
  return SIM_OK;
}

int sim_probe_fma(void* scratch, size_t scratch_bytes, void* hip_stream, double* tflops) {
  const size_t need = (size_t)PROBE_FMA_BLOCKS * PROBE_FMA_THREADS * sizeof(float);
  if (!scratch || !tflops) return fail(SIM_E_ARG, "sim_probe_fma: null argument");
  if (scratch_bytes < need) return fail(SIM_E_ARG, "sim_probe_fma: scratch smaller than sim_probe_fma_bytes()");
  hipStream_t s = (hipStream_t)hip_stream;
  float ms = 0.f;
  const int rc = probe_time([&] {
    hipLaunchKernelGGL(k_probe_fma, dim3(PROBE_FMA_BLOCKS), dim3(PROBE_FMA_THREADS), 0, s, (float*)scratch, 0.999999f, 1e-7f);
  }, s, &ms);
  if (rc) return rc;
  const double flops = 2.0 * 8.0 * PROBE_FMA_ITERS * (double)PROBE_FMA_BLOCKS * PROBE_FMA_THREADS;
  *tflops = flops / (ms * 1e-3) / 1e12;
  g_err.clear();
  return SIM_OK;
}

size_t sim_probe_fma_bytes(void) { return (size_t)PROBE_FMA_BLOCKS * PROBE_FMA_THREADS * sizeof(float); }

int sim_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream, double* gbs) {
  if (!src || !dst || !gbs) return fail(SIM_E_ARG, "sim_probe_copy: null argument");
  if (bytes < 16 || bytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
    return fail(SIM_E_ARG, "sim_probe_copy: bytes and both pointers must be multiples of 16");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t n = bytes / 16;
  float ms = 0.f;
  const int rc = probe_time([&] {
    hipLaunchKernelGGL(k_probe_copy, dim3(4096), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n);
  }, s, &ms);
  if (rc) return rc;
  *gbs = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
  g_err.clear();
  return SIM_OK;
}

// ======================================================================= learning-episode update
static int learn_launch(float, const LearnAdamT<float>& A, void* s) { return sim_l32::launch_adam(A, s); }
static int learn_launch(double, const LearnAdamT<double>& A, void* s) { return sim_l64::launch_adam(A, s); }
static int soft_launch(float* t, const float* o, long n, double a, void* s) { return sim_l32::launch_soft_update(t, o, n, (float)a, s); }
static int soft_launch(double* t, const double* o, long n, double a, void* s) { return sim_l64::launch_soft_update(t, o, n, a, s); }
static int td_launch(const float* r, const float* v, const uint8_t* d, int h, int N, double g, double l, float* out,
                     void* s) {
  return sim_l32::launch_td_lambda(r, v, d, h, N, (float)g, (float)l, out, s);
}
static int td_launch(const double* r, const double* v, const uint8_t* d, int h, int N, double g, double l, double* out,
                     void* s) {
  return sim_l64::launch_td_lambda(r, v, d, h, N, g, l, out, s);
}
static int cv_launch(const ThetaArgsT<float>& T, float* out, void* s) { return sim_l32::launch_critic_values(T, out, s); }
static int cv_launch(const ThetaArgsT<double>& T, double* out, void* s) { return sim_l64::launch_critic_values(T, out, s); }
static int cf_launch(const CriticFitT<float>& F, void* s) { return sim_l32::launch_critic_fit(F, s); }
static int cf_launch(const CriticFitT<double>& F, void* s) { return sim_l64::launch_critic_fit(F, s); }

template <typename T>
static int adam_impl(void* const* tensors, const size_t* sizes, int n, const void* grad, void* m, void* v, int step,
                     double lr, double b1, double b2, double eps, void* stream) {
  LearnAdamT<T> A;
  std::memset(&A, 0, sizeof(A));
  A.n = n;
  for (int i = 0; i < n; ++i) {
    A.p[i] = static_cast<T*>(tensors[i]);
    A.size[i] = (long)sizes[i];
  }
  A.g = static_cast<const T*>(grad); A.m = static_cast<T*>(m); A.v = static_cast<T*>(v);
  A.lr = (T)lr; A.b1 = (T)b1; A.b2 = (T)b2; A.eps = (T)eps;
  A.bc1 = (T)(1.0 - std::pow(b1, (double)step));
  A.bc2 = (T)(1.0 - std::pow(b2, (double)step));
  if (learn_launch(T(), A, stream)) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

extern "C" int sim_adam_step(void* const* tensors, const size_t* sizes, int n_tensors, const void* grad, void* m,
                             void* v, int step, double lr, double beta1, double beta2, double eps, int precision,
                             void* hip_stream) {
  if (!tensors || !sizes || !grad || !m || !v || n_tensors < 1 || n_tensors > SIM_MAX_TENSORS)
    return fail(SIM_E_ARG, "sim_adam_step: null pointer or tensor count outside 1..SIM_MAX_TENSORS");
  for (int i = 0; i < n_tensors; ++i)
    if (!tensors[i] || sizes[i] == 0) return fail(SIM_E_ARG, "sim_adam_step: null or empty tensor");
  if (step < 1) return fail(SIM_E_ARG, "sim_adam_step: step counts from 1");
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return fail(SIM_E_ARG, "sim_adam_step: need lr >= 0, 0 <= beta < 1, eps > 0");
  if (precision == SIM_PREC_FP32)
    return adam_impl<float>(tensors, sizes, n_tensors, grad, m, v, step, lr, beta1, beta2, eps, hip_stream);
  if (precision == SIM_PREC_FP64)
    return adam_impl<double>(tensors, sizes, n_tensors, grad, m, v, step, lr, beta1, beta2, eps, hip_stream);
  return fail(SIM_E_ARG, "sim_adam_step: unknown precision");
}

extern "C" int sim_soft_update(void* const* target, const void* const* online, const size_t* sizes, int n_tensors,
                               double alpha, int precision, void* hip_stream) {
  if (!target || !online || !sizes || n_tensors < 1 || n_tensors > SIM_MAX_TENSORS)
    return fail(SIM_E_ARG, "sim_soft_update: null pointer or tensor count outside 1..SIM_MAX_TENSORS");
  for (int i = 0; i < n_tensors; ++i)
    if (!target[i] || !online[i] || sizes[i] == 0) return fail(SIM_E_ARG, "sim_soft_update: null or empty tensor");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(SIM_E_ARG, "sim_soft_update: alpha outside [0, 1]");
  if (precision != SIM_PREC_FP32 && precision != SIM_PREC_FP64) return fail(SIM_E_ARG, "sim_soft_update: unknown precision");
  int bad = 0;
  for (int i = 0; i < n_tensors; ++i) {
    if (precision == SIM_PREC_FP32)
      bad |= soft_launch(static_cast<float*>(target[i]), static_cast<const float*>(online[i]), (long)sizes[i], alpha, hip_stream);
    else
      bad |= soft_launch(static_cast<double*>(target[i]), static_cast<const double*>(online[i]), (long)sizes[i], alpha, hip_stream);
  }
  if (bad) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

extern "C" int sim_td_lambda(const void* rewards, const void* values, const uint8_t* done, int h, int n_envs,
                             double gamma, double lambda, void* targets, int precision, void* hip_stream) {
  if (!rewards || !values || !targets || h < 1 || n_envs < 1) return fail(SIM_E_ARG, "sim_td_lambda: null pointer or empty window");
  if (!(gamma >= 0.0 && gamma <= 1.0) || !(lambda >= 0.0 && lambda <= 1.0))
    return fail(SIM_E_ARG, "sim_td_lambda: gamma and lambda must lie in [0, 1]");
  int bad;
  if (precision == SIM_PREC_FP32)
    bad = td_launch(static_cast<const float*>(rewards), static_cast<const float*>(values), done, h, n_envs, gamma, lambda,
                    static_cast<float*>(targets), hip_stream);
  else if (precision == SIM_PREC_FP64)
    bad = td_launch(static_cast<const double*>(rewards), static_cast<const double*>(values), done, h, n_envs, gamma,
                    lambda,
                    static_cast<double*>(targets), hip_stream);
  else
    return fail(SIM_E_ARG, "sim_td_lambda: unknown precision");
  if (bad) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

extern "C" int sim_obs_stats_update(const void* obs, long rows, int dim, double count, void* mean, void* var,
                                    void* inv_std, double eps, int precision, void* hip_stream) {
  if (!obs || !mean || !var || !inv_std || rows < 1 || dim < 1)
    return fail(SIM_E_ARG, "sim_obs_stats_update: null pointer or empty batch");
  if (!(count >= 0.0) || !(eps >= 0.0)) return fail(SIM_E_ARG, "sim_obs_stats_update: need count >= 0 and eps >= 0");
  int bad;
  if (precision == SIM_PREC_FP32)
    bad = sim_l32::launch_obs_stats(static_cast<const float*>(obs), rows, dim, count, static_cast<float*>(mean),
                                    static_cast<float*>(var), static_cast<float*>(inv_std), eps, hip_stream);
  else if (precision == SIM_PREC_FP64)
    bad = sim_l64::launch_obs_stats(static_cast<const double*>(obs), rows, dim, count, static_cast<double*>(mean),
                                    static_cast<double*>(var), static_cast<double*>(inv_std), eps, hip_stream);
  else
    return fail(SIM_E_ARG, "sim_obs_stats_update: unknown precision");
  if (bad) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

// workspace of the critic calls: x [rows][od], y [rows], V [rows], H[1..nl-1] [rows][dims],
// d0 / d1 [rows][max width], split partials, the flat gradient
#define CRITIC_SPLITS 32
struct CriticWs {
  size_t x, y, v, h[SIM_MAXL], d0, d1, part, grad, total;
  size_t yn[SIM_MAXL], st, lnpart;   // with layer normalisation
};
static CriticWs critic_ws(const SimOptions& o, int rows, size_t e) {
  CriticWs w = {};
  const int L = o.critic_layers;
  int maxd = 0;
  size_t maxpart = 0, nparams = 0;
  for (int l = 0; l <= L; ++l) maxd = std::max(maxd, o.critic_dims[l]);
  for (int l = 0; l < L; ++l) {
    maxpart = std::max(maxpart, (size_t)o.critic_dims[l + 1] * (o.critic_dims[l] + 1));
    nparams += (size_t)o.critic_dims[l + 1] * (o.critic_dims[l] + 1);
    if (o.layer_norm && l + 1 < L) nparams += 2 * (size_t)o.critic_dims[l + 1];
  }
  size_t off = 0;
  w.x = off; off = align256(off + (size_t)rows * o.critic_dims[0] * e);
  w.y = off; off = align256(off + (size_t)rows * e);
  w.v = off; off = align256(off + (size_t)rows * e);
  for (int l = 1; l < L; ++l) { w.h[l] = off; off = align256(off + (size_t)rows * o.critic_dims[l] * e); }
  w.d0 = off; off = align256(off + (size_t)rows * maxd * e);
  w.d1 = off; off = align256(off + (size_t)rows * maxd * e);
  w.part = off; off = align256(off + (size_t)CRITIC_SPLITS * maxpart * e);
  w.grad = off; off = align256(off + nparams * e);
  if (o.layer_norm && L > 1) {
    // the normalised hidden layers, their per-row statistics, the gain / bias partials
    for (int l = 1; l < L; ++l) { w.yn[l] = off; off = align256(off + (size_t)rows * o.critic_dims[l] * e); }
    w.st = off; off = align256(off + (size_t)rows * 2 * (L - 1) * e);
    w.lnpart = off; off = align256(off + (size_t)SIM_LN_BLOCKS * 2 * maxd * e);
  }
  w.total = off;
  return w;
}

extern "C" size_t sim_critic_workspace_bytes(const SimHandle* h, int rows) {
  if (check_handle(const_cast<SimHandle*>(h)) || rows < 1) return 0;
  const size_t e = (h->opt.precision == SIM_PREC_FP64) ? 8 : 4;
  return critic_ws(h->opt, rows, e).total;
}

template <typename T>
static void critic_theta_args(const SimHandle* h, const CriticWs& w, char* ws, const void* const* cw, const void* const* cb,
                              const void* const* clg, const void* const* clb, int rows, ThetaArgsT<T>& P) {
  const SimOptions& o = h->opt;
  std::memset(&P, 0, sizeof(P));
  P.M = rows;
  P.nl = o.critic_layers;
  for (int l = 0; l <= o.critic_layers; ++l) P.dims[l] = o.critic_dims[l];
  P.splits = CRITIC_SPLITS;
  const bool ln = o.layer_norm && o.critic_layers > 1;
  long off = 0;
  for (int l = 0; l < o.critic_layers; ++l) {
    P.W[l] = static_cast<const T*>(cw[l]);
    P.b[l] = static_cast<const T*>(cb[l]);
    P.off_w[l] = off;
    off += (long)o.critic_dims[l] * o.critic_dims[l + 1];
    P.off_b[l] = off;
    off += o.critic_dims[l + 1];
    if (ln && l + 1 < o.critic_layers) {
      // the hidden layer's normalisation gain and bias follow its W, b
      P.lng[l] = static_cast<const T*>(clg[l]);
      P.lnb[l] = static_cast<const T*>(clb[l]);
      P.off_g[l] = off;
      off += o.critic_dims[l + 1];
      P.off_beta[l] = off;
      off += o.critic_dims[l + 1];
    }
    if (l >= 1) P.H[l] = reinterpret_cast<T*>(ws + w.h[l]);
  }
  if (ln) {
    P.ln = 1;
    P.ln_eps = (T)1e-5;
    P.st = reinterpret_cast<T*>(ws + w.st);
    P.ldst = 2 * (o.critic_layers - 1);
    for (int l = 1; l < o.critic_layers; ++l) P.Y[l] = reinterpret_cast<T*>(ws + w.yn[l]);
    P.lnpart = reinterpret_cast<T*>(ws + w.lnpart);
    P.ln_blocks = SIM_LN_BLOCKS;
  }
  P.d0 = reinterpret_cast<T*>(ws + w.d0);
  P.d1 = reinterpret_cast<T*>(ws + w.d1);
  P.part = reinterpret_cast<T*>(ws + w.part);
  P.out = reinterpret_cast<T*>(ws + w.grad);
}

template <typename T>
static int critic_values_impl(SimHandle* h, const void* obs, int rows, const void* const* cw, const void* const* cb,
                              const void* const* clg, const void* const* clb, const void* mean, const void* inv_std,
                              void* values, void* workspace, void* stream) {
  const CriticWs w = critic_ws(h->opt, rows, sizeof(T));
  ThetaArgsT<T> P;
  critic_theta_args<T>(h, w, static_cast<char*>(workspace), cw, cb, clg, clb, rows, P);
  P.x0 = static_cast<const T*>(obs);
  P.x_shift = static_cast<const T*>(mean);
  P.x_scale = static_cast<const T*>(inv_std);
  if (cv_launch(P, static_cast<T*>(values), stream)) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

// the checks and the launch of sim_critic_values and sim_critic_values_ln
static int critic_values_checked(SimHandle* h, const char* fn, const void* obs, int rows, const void* const* critic_w,
                                 const void* const* critic_b, const void* const* ln_g, const void* const* ln_b,
                                 const void* obs_mean, const void* obs_inv_std, void* values, void* workspace,
                                 size_t workspace_bytes, void* hip_stream) {
  const std::string f(fn);
  if (!obs || !values || !critic_w || !critic_b || rows < 1) return fail(SIM_E_ARG, f + ": null pointer or no rows");
  for (int l = 0; l < h->opt.critic_layers; ++l)
    if (!critic_w[l] || !critic_b[l]) return fail(SIM_E_ARG, f + ": null critic weights");
  if (h->opt.layer_norm)
    for (int l = 0; l + 1 < h->opt.critic_layers; ++l)
      if (!ln_g || !ln_b || !ln_g[l] || !ln_b[l]) return fail(SIM_E_ARG, f + ": null layer-normalisation gain or bias");
  if ((obs_mean != nullptr) != (obs_inv_std != nullptr))
    return fail(SIM_E_ARG, f + ": observation normalisation needs both obs_mean and obs_inv_std");
  if (!workspace || workspace_bytes < sim_critic_workspace_bytes(h, rows))
    return fail(SIM_E_WORKSPACE, f + ": workspace smaller than sim_critic_workspace_bytes()");
  return (h->opt.precision == SIM_PREC_FP64)
             ? critic_values_impl<double>(h, obs, rows, critic_w, critic_b, ln_g, ln_b, obs_mean, obs_inv_std, values,
                                          workspace, hip_stream)
             : critic_values_impl<float>(h, obs, rows, critic_w, critic_b, ln_g, ln_b, obs_mean, obs_inv_std, values,
                                         workspace, hip_stream);
}

extern "C" int sim_critic_values(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                                 const void* const* critic_b, const void* obs_mean, const void* obs_inv_std,
                                 void* values, void* workspace, size_t workspace_bytes, void* hip_stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->opt.layer_norm)
    return fail(SIM_E_UNSUPPORTED, "sim_critic_values: a handle with layer normalisation takes sim_critic_values_ln");
  return critic_values_checked(h, "sim_critic_values", obs, rows, critic_w, critic_b, nullptr, nullptr, obs_mean,
                               obs_inv_std, values, workspace, workspace_bytes, hip_stream);
}

extern "C" int sim_critic_values_ln(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                                    const void* const* critic_b, const void* const* critic_ln_g,
                                    const void* const* critic_ln_b, const void* obs_mean, const void* obs_inv_std,
                                    void* values, void* workspace, size_t workspace_bytes, void* hip_stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  return critic_values_checked(h, "sim_critic_values_ln", obs, rows, critic_w, critic_b, critic_ln_g, critic_ln_b,
                               obs_mean, obs_inv_std, values, workspace, workspace_bytes, hip_stream);
}

// the critic's hidden-layer activations [rows][dims[l]] (l = 1 .. L-1), one after the other
static size_t critic_hidden_bytes(const SimOptions& o, int rows, size_t e, size_t* off) {
  size_t total = 0;
  for (int l = 1; l < o.critic_layers; ++l) {
    if (off) off[l] = total;
    total = align256(total + (size_t)rows * o.critic_dims[l] * e);
  }
  return total;
}

template <typename T>
static int critic_values_noalloc_impl(SimHandle* h, const void* obs, int rows, const void* const* cw,
                                      const void* const* cb, const void* mean, const void* inv_std, void* values,
                                      char* scr, void* stream) {
  const SimOptions& o = h->opt;
  size_t off[SIM_MAXL] = {};
  critic_hidden_bytes(o, rows, sizeof(T), off);
  ThetaArgsT<T> P;
  std::memset(&P, 0, sizeof(P));
  P.M = rows;
  P.nl = o.critic_layers;
  for (int l = 0; l <= o.critic_layers; ++l) P.dims[l] = o.critic_dims[l];
  for (int l = 0; l < o.critic_layers; ++l) {
    P.W[l] = static_cast<const T*>(cw[l]);
    P.b[l] = static_cast<const T*>(cb[l]);
    if (l >= 1) P.H[l] = reinterpret_cast<T*>(scr + off[l]);
  }
  P.x0 = static_cast<const T*>(obs);
  P.x_shift = static_cast<const T*>(mean);
  P.x_scale = static_cast<const T*>(inv_std);
  if (cv_launch(P, static_cast<T*>(values), stream)) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

extern "C" int sim_critic_values_noalloc(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                                         const void* const* critic_b, const void* obs_mean, const void* obs_inv_std,
                                         void* values, void* hip_stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->opt.layer_norm)
    return fail(SIM_E_UNSUPPORTED, "sim_critic_values_noalloc: a handle with layer normalisation takes sim_critic_values_ln (with a workspace)");
  if (!obs || !values || !critic_w || !critic_b || rows < 1)
    return fail(SIM_E_ARG, "sim_critic_values_noalloc: null pointer or no rows");
  for (int l = 0; l < h->opt.critic_layers; ++l)
    if (!critic_w[l] || !critic_b[l]) return fail(SIM_E_ARG, "sim_critic_values_noalloc: null critic weights");
  if ((obs_mean != nullptr) != (obs_inv_std != nullptr))
    return fail(SIM_E_ARG, "sim_critic_values_noalloc: observation normalisation needs both obs_mean and obs_inv_std");
  const size_t e = h->elem;
  const size_t per_row = critic_hidden_bytes(h->opt, 1, e, nullptr);
  if (critic_hidden_bytes(h->opt, rows, e, nullptr) > SIM_NOALLOC_SCRATCH_BYTES)
    return fail(SIM_E_WORKSPACE, "sim_critic_values_noalloc: " + std::to_string(rows) + " rows need more than the " +
                                     std::to_string(SIM_NOALLOC_SCRATCH_BYTES >> 20) + " MiB static scratch (about " +
                                     std::to_string(per_row ? SIM_NOALLOC_SCRATCH_BYTES / per_row : 0) +
                                     " rows of this critic fit)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_E_HIP, "sim_critic_values_noalloc: hipGetDevice failed");
  char* scr = static_cast<char*>(scratch_on_device(dev));
  if (!scr) return fail(SIM_E_HIP, "sim_critic_values_noalloc: hipGetSymbolAddress of the static scratch failed");
  return (h->opt.precision == SIM_PREC_FP64)
             ? critic_values_noalloc_impl<double>(h, obs, rows, critic_w, critic_b, obs_mean, obs_inv_std, values, scr,
                                                  hip_stream)
             : critic_values_noalloc_impl<float>(h, obs, rows, critic_w, critic_b, obs_mean, obs_inv_std, values, scr,
                                                 hip_stream);
}

template <typename T>
static int critic_fit_impl(SimHandle* h, const SimCriticFitIO* io, void* stream) {
  const CriticWs w = critic_ws(h->opt, io->rows, sizeof(T));
  char* ws = static_cast<char*>(io->workspace);
  CriticFitT<T> F;
  std::memset(&F, 0, sizeof(F));
  critic_theta_args<T>(h, w, ws, io->critic_w, io->critic_b, io->critic_ln_g, io->critic_ln_b, io->rows, F.G);
  F.obs = static_cast<const T*>(io->obs);
  F.obs_mean = static_cast<const T*>(io->obs_mean);
  F.obs_inv_std = static_cast<const T*>(io->obs_inv_std);
  F.targets = static_cast<const T*>(io->targets);
  F.perm = io->perm;
  F.rows = io->rows; F.n_iter = io->n_iter; F.n_mb = io->n_minibatch;
  F.x = reinterpret_cast<T*>(ws + w.x);
  F.y = reinterpret_cast<T*>(ws + w.y);
  F.vbuf = reinterpret_cast<T*>(ws + w.v);
  for (int l = 0; l < h->opt.critic_layers; ++l) {
    F.W[l] = static_cast<T*>(io->critic_w[l]);
    F.bvec[l] = static_cast<T*>(io->critic_b[l]);
    if (F.G.ln && l + 1 < h->opt.critic_layers) {
      F.lng[l] = static_cast<T*>(io->critic_ln_g[l]);
      F.lnb[l] = static_cast<T*>(io->critic_ln_b[l]);
    }
  }
  F.m = static_cast<T*>(io->adam_m);
  F.v = static_cast<T*>(io->adam_v);
  F.adam_step = io->adam_step;
  F.lr = (T)io->lr; F.b1 = (T)io->beta1; F.b2 = (T)io->beta2; F.eps = (T)io->eps;
  F.loss_out = static_cast<T*>(io->loss_out);
  if (cf_launch(F, stream)) return launch_failed();
  g_err.clear();
  return SIM_OK;
}

extern "C" int sim_critic_fit(SimHandle* h, const SimCriticFitIO* io, void* hip_stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!io || !io->obs || !io->targets || !io->perm || !io->adam_m || !io->adam_v)
    return fail(SIM_E_ARG, "sim_critic_fit: null pointer");
  if (h->opt.layer_norm)
    for (int l = 0; l + 1 < h->opt.critic_layers; ++l)
      if (!io->critic_ln_g[l] || !io->critic_ln_b[l])
        return fail(SIM_E_ARG, "sim_critic_fit: null layer-normalisation gain or bias");
  if (io->rows < 1 || io->n_iter < 1 || io->n_minibatch < 1 || io->n_minibatch > io->rows)
    return fail(SIM_E_ARG, "sim_critic_fit: need rows >= 1, n_iter >= 1, 1 <= n_minibatch <= rows");
  for (int l = 0; l < h->opt.critic_layers; ++l)
    if (!io->critic_w[l] || !io->critic_b[l]) return fail(SIM_E_ARG, "sim_critic_fit: null critic weights");
  if (io->adam_step < 0 || !(io->lr >= 0.0) || !(io->beta1 >= 0.0 && io->beta1 < 1.0) ||
      !(io->beta2 >= 0.0 && io->beta2 < 1.0) || !(io->eps > 0.0))
    return fail(SIM_E_ARG, "sim_critic_fit: need adam_step >= 0, lr >= 0, 0 <= beta < 1, eps > 0");
  if ((io->obs_mean != nullptr) != (io->obs_inv_std != nullptr))
    return fail(SIM_E_ARG, "sim_critic_fit: observation normalisation needs both obs_mean and obs_inv_std");
  if (!io->workspace || io->workspace_bytes < sim_critic_workspace_bytes(h, io->rows))
    return fail(SIM_E_WORKSPACE, "sim_critic_fit: workspace smaller than sim_critic_workspace_bytes()");
  return (h->opt.precision == SIM_PREC_FP64) ? critic_fit_impl<double>(h, io, hip_stream)
                                             : critic_fit_impl<float>(h, io, hip_stream);
}

// ---------------------------------------------------------------- phase profile readout
extern "C" int sim_phase_profile(unsigned long long* out, int n, int reset) {
#ifdef SIM_PHASE_PROFILE
  if (!out || n < 0 || n > SIM_NPHASE) return fail(SIM_E_ARG, "sim_phase_profile: out and 0 <= n <= SIM_NPHASE");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_E_HIP, "hipGetDevice failed");
  unsigned long long* p = phase_on_device(dev);
  if (!p) return fail(SIM_E_HIP, "sim_phase_profile: hipGetSymbolAddress failed");
  if (hipDeviceSynchronize() != hipSuccess) return fail(SIM_E_HIP, "hipDeviceSynchronize failed");
  if (n > 0 && hipMemcpy(out, p, n * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SIM_E_HIP, "hipMemcpy failed");
  if (reset && hipMemset(p, 0, SIM_NPHASE * sizeof(unsigned long long)) != hipSuccess)
    return fail(SIM_E_HIP, "hipMemset failed");
  if (reset && hipDeviceSynchronize() != hipSuccess) return fail(SIM_E_HIP, "hipDeviceSynchronize failed");
  return SIM_NPHASE;
#else
  (void)out; (void)n; (void)reset;
  return fail(SIM_E_UNSUPPORTED, "sim_phase_profile: this library was built without -DSIM_PHASE_PROFILE");
#endif
}
