// Window kernels (persistent and plain per-step paths) and their launchers, for one
// arithmetic type.  Included inside the namespace of one precision by several translation
// units, which compile in parallel: SIM_EMIT_MAIN emits the full and muscle layouts' windows,
// the plain path, the weight preparation, the window loss and the group launcher;
// SIM_EMIT_COMPACT the compact layouts' windows; SIM_EMIT_GROUP_FWD / SIM_EMIT_GROUP_ADJ the
// forward / adjoint mixed-morphology group kernel.
#ifndef SIM_EMIT_MAIN
#define SIM_EMIT_MAIN 0
#endif
#ifndef SIM_EMIT_COMPACT
#define SIM_EMIT_COMPACT 0
#endif
#ifndef SIM_EMIT_GROUP_FWD
#define SIM_EMIT_GROUP_FWD 0
#endif
#ifndef SIM_EMIT_GROUP_ADJ
#define SIM_EMIT_GROUP_ADJ 0
#endif

// launchers defined by another unit of the same precision
int launch_compact(const WinArgs& A, int adjoint, int nv, int lanes, void* stream);
void launch_window_loss(const WinArgs& A, hipStream_t s);
int launch_group_fwd(const GroupArgs& G, size_t lds_bytes, hipStream_t s);
int launch_group_adj(const GroupArgs& G, size_t lds_bytes, hipStream_t s);
int prepare_group_fwd(size_t lds_bytes);
int prepare_group_adj(size_t lds_bytes);

// ======================================================================= device helpers
template <int LN>
__device__ __forceinline__ bool all_finite_env(bool ok) {
  return grp_all<LN>(ok);
}

template <class L>
__device__ __forceinline__ void load_state(const Scal* __restrict__ m, L& E, const real* s, int ln) {
  int nq = m->nq, nv = m->nv;
  for (int i = ln; i < nq; i += L::kLanes) E.q[i] = s[i];
  for (int i = ln; i < nv; i += L::kLanes) E.qd[i] = s[nq + i];
  if (m->has_last_action)
    for (int i = ln; i < m->na; i += L::kLanes) E.a[i] = s[nq + nv + i];
  else
    for (int i = ln; i < L::kMaxA; i += L::kLanes) E.a[i] = RL(0.0);
  if constexpr (L::kMtu > 0) {
    const int o = nq + nv + (m->has_last_action ? m->na : 0);
    for (int i = ln; i < m->n_mtu; i += L::kLanes) E.act[i] = s[o + i];
  }
  __syncthreads();
}

// checkpoint of the dynamic state: [q | qd | act] (nck values)
template <class L>
__device__ __forceinline__ void store_qqd(const Scal* __restrict__ m, const L& E, real* dst, int ln) {
  int nq = m->nq, nv = m->nv;
  for (int i = ln; i < nq; i += L::kLanes) dst[i] = E.q[i];
  for (int i = ln; i < nv; i += L::kLanes) dst[nq + i] = E.qd[i];
  if constexpr (L::kMtu > 0)
    for (int i = ln; i < m->n_mtu; i += L::kLanes) dst[nq + nv + i] = E.act[i];
}

template <class L>
__device__ __forceinline__ void load_qqd(const Scal* __restrict__ m, L& E, const real* src, int ln) {
  int nq = m->nq, nv = m->nv;
  for (int i = ln; i < nq; i += L::kLanes) E.q[i] = src[i];
  for (int i = ln; i < nv; i += L::kLanes) E.qd[i] = src[nq + i];
  if constexpr (L::kMtu > 0)
    for (int i = ln; i < m->n_mtu; i += L::kLanes) E.act[i] = src[nq + nv + i];
  __syncthreads();
}

// observation normalisation with running statistics (Sec. 3.3): the networks read
// o_hat = (o - mean) * inv_std, so the observation adjoint is o_hat_bar * inv_std
template <int LN>
__device__ __forceinline__ void obs_normalize(const WinArgs& A, const Scal* __restrict__ m, real* o, int ln) {
  if (!A.obs_mean) return;
  for (int i = ln; i < m->od; i += LN) o[i] = (o[i] - A.obs_mean[i]) * A.obs_inv_std[i];
  __syncthreads();
}
template <int LN>
__device__ __forceinline__ void obs_adjoint_scale(const WinArgs& A, const Scal* __restrict__ m, real* ob, int ln) {
  if (!A.obs_mean) return;
  for (int i = ln; i < m->od; i += LN) ob[i] *= A.obs_inv_std[i];
  __syncthreads();
}

// observation, action and reward at the start of frame t (state in E.q/E.qd, previous
// action in E.a); leaves a_t in E.a.
template <class L>
__device__ __forceinline__ void frame_begin(const WinArgs& A, const Scal* __restrict__ m, L& E,
                                            int env, int t, int ln) {
  const int N = A.N, od = m->od, na = m->na;
  task_obs<L::kLanes>(m, E.q, E.qd, E.a, E.act, E.obs, ln);
  real* ob = A.obs + ((size_t)t * N + env) * od;
  for (int i = ln; i < od; i += L::kLanes) ob[i] = E.obs[i];
  SIM_PHASE(E, PH_FB_OBS);
  if (A.closed_loop) {
    obs_normalize<L::kLanes>(A, m, E.obs, ln);
    mlp_forward<L::kLanes>(A.actor, E.obs, E.h0, E.h1, E.y, E.xb16, ln, E.gb, E.lnst);
    SIM_PHASE(E, PH_FB_MLP);
    // keep the hidden activations for the adjoint's input VJP (at most two hidden layers; with
    // layer normalisation the ELU outputs and then each hidden layer's mean and inverse
    // deviation)
    {
      real* hs = A.hid + ((size_t)t * N + env) * A.hid_w;
      const int d1 = A.actor.nl > 1 ? A.actor.dims[1] : 0, d2 = A.actor.nl > 2 ? A.actor.dims[2] : 0;
      for (int i = ln; i < d1; i += L::kLanes) hs[i] = E.h0[i];
      for (int i = ln; i < d2; i += L::kLanes) hs[d1 + i] = E.h1[i];
      if (A.actor.ln && ln < 2 * (A.actor.nl - 1)) hs[d1 + d2 + ln] = E.lnst[ln];
    }
    if (A.noise) {
      // stochastic policy, reparameterised (Sec. 3.3): y = mu(o) + exp(log_std) * eps
      const real* ep = A.noise + ((size_t)t * N + env) * na;
      for (int i = ln; i < na; i += L::kLanes) E.a[i] = squash(m, m_fma(m_exp(A.log_std[i]), ep[i], E.y[i]));
    } else {
      for (int i = ln; i < na; i += L::kLanes) E.a[i] = squash(m, E.y[i]);
    }
  } else {
    const real* ai = A.actions_in + ((size_t)t * N + env) * na;
    for (int i = ln; i < na; i += L::kLanes) E.a[i] = ai[i];
  }
  __syncthreads();
  real r = task_reward(m, E.q, E.qd, E.a, ln);
  if (ln == 0) A.rewards[(size_t)t * N + env] = r;
  real* ao = A.actions + ((size_t)t * N + env) * na;
  for (int i = ln; i < na; i += L::kLanes) ao[i] = E.a[i];
  __syncthreads();
}

template <class L>
__device__ __forceinline__ void window_end(const WinArgs& A, const Scal* __restrict__ m, L& E,
                                           int env, int ln) {
  const int N = A.N, od = m->od, ns = m->ns, nq = m->nq, nv = m->nv, na = m->na;
  task_obs<L::kLanes>(m, E.q, E.qd, E.a, E.act, E.obs, ln);
  real* ob = A.obs + ((size_t)A.h * N + env) * od;
  for (int i = ln; i < od; i += L::kLanes) ob[i] = E.obs[i];
  obs_normalize<L::kLanes>(A, m, E.obs, ln);
  mlp_forward<L::kLanes>(A.critic, E.obs, E.h0, E.h1, E.y, E.xb16, ln, E.gb, E.lnst);
  if (ln == 0) A.value[env] = E.y[0];
  real* so = A.s_h + (size_t)env * ns;
  bool ok = true;
  for (int i = ln; i < nq; i += L::kLanes) { so[i] = E.q[i]; ok = ok && m_isfinite(E.q[i]); }
  for (int i = ln; i < nv; i += L::kLanes) { so[nq + i] = E.qd[i]; ok = ok && m_isfinite(E.qd[i]); }
  if (m->has_last_action)
    for (int i = ln; i < na; i += L::kLanes) so[nq + nv + i] = E.a[i];
  if constexpr (L::kMtu > 0) {
    const int o = nq + nv + (m->has_last_action ? na : 0);
    for (int i = ln; i < m->n_mtu; i += L::kLanes) { so[o + i] = E.act[i]; ok = ok && m_isfinite(E.act[i]); }
  }
  bool all = all_finite_env<L::kLanes>(ok);
  if (ln == 0 && A.nonfinite) A.nonfinite[env] = all ? 0 : 1;
}

// Launch forms a window kernel is compiled for: any (chosen per launch from the arguments, as in
// the group kernels), or one fixed form, so that the kernel carries only that form's code and
// registers.
enum { KP_ANY = -1, KP_TAPE = 0, KP_FC = 1, KP_CKPT = 2 };

// ======================================================================= persistent forward
// One environment's forward window (the wavefront owns env; E is its LDS).  PATH: KP_TAPE,
// KP_CKPT (checkpoints, with or without the factor cache) or KP_ANY.
template <int NV, class L, int PATH = KP_ANY>
__device__ __forceinline__ void window_fwd_body(const WinArgs& A, int env, L& E) {
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int ln = grp_lane<L::kLanes>();
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nqv = m->nck, N = A.N;
  load_state(m, E, A.s0 + (size_t)env * m->ns, ln);
  const TapeMap<L> TM = tape_map<L>(m, ln);
  const FcMap<L> FM = fc_map<L>(m, ln);
#ifdef SIM_PHASE_PROFILE
  phase_start<L::kLanes>(E.prof);
#endif
  Chol C;
  int nfb = 0, nadh = 0;
  int t0 = 0;   // first frame of the current discount segment (early termination)
  for (int t = 0; t < A.h; ++t) {
    frame_begin(A, m, E, env, t, ln);
    SIM_PHASE(E, PH_FRAME_BEGIN);
    for (int sub = 0; sub < S; ++sub) {
      int gi = t * S + sub;
      int fb;
      if (PATH == KP_TAPE || (PATH == KP_ANY && A.tape_full)) {
        // the tape entry holds the pre-substep state and the linearisation
        substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
        tape_store<NV>(TM, E, C, fb, ln, A.tape + ((size_t)gi * N + env) * A.tape_ws);
        commit_substep(m, E, ln);
      } else {
        if (gi % A.k == 0) {
          store_qqd(m, E, A.ckpt + ((size_t)(gi / A.k) * N + env) * nqv, ln);
          SIM_PHASE(E, PH_CKPT);
        }
        substep_forward<NV>(m, E, jr, cr, ln, C, true, fb);
        if constexpr (L::kMtu == 0)
          if (A.fc) fc_store<NV>(m, FM, E, C, fb, ln, A.fc + ((size_t)gi * N + env) * A.fc_ws,
                                 A.fcq + ((size_t)gi * N + env) * m->nv);
      }
      nfb += fb;
      nadh += E.nadh;
    }
    if (m->term) {
      // early termination: the frame ended with the root below the height; the env restarts
      // from its reset state, a constant, and its discount from the next frame
      const int done = (E.q[2] < m->term_h) ? 1 : 0;
      if (ln == 0) {
        A.done_ws[(size_t)t * N + env] = (uint8_t)done;
        if (A.done_out) A.done_out[(size_t)t * N + env] = (uint8_t)done;
        A.seg_ws[(size_t)t * N + env] = t0;
      }
      if (done) {
        load_state(m, E, A.reset + (size_t)env * m->ns, ln);
        t0 = t + 1;
      }
      SIM_PHASE(E, PH_TERM);
    }
  }
  if (m->term && ln == 0) A.seg_ws[(size_t)A.h * N + env] = t0;
  window_end(A, m, E, env, ln);
  if (ln == 0 && A.fallback) A.fallback[env] = nfb;
  if (ln == 0 && A.adhesive) A.adhesive[env] = nadh;
#ifdef SIM_PHASE_PROFILE
  SIM_PHASE(E, PH_WINDOW_END);
  phase_flush<L::kLanes>(E.prof, A.prof);
#endif
}

// ======================================================================= persistent adjoint
// terminal seed: s_bar(h) = -gamma^h scale (d obs/d s)^T dV/d obs  (+ optional upstream)
template <class L>
__device__ __forceinline__ void adjoint_seed(const WinArgs& A, const Scal* __restrict__ m, L& E,
                                             int env, int ln) {
  const int ns = m->ns, nq = m->nq, nv = m->nv, na = m->na, od = m->od;
  const real* sh = A.s_h_in + (size_t)env * ns;
  load_state(m, E, sh, ln);
  for (int i = ln; i < L::kQ; i += L::kLanes) E.qb[i] = RL(0.0);
  for (int i = ln; i < L::kV; i += L::kLanes) E.qdb[i] = RL(0.0);
  for (int i = ln; i < L::kMaxA; i += L::kLanes) E.abar[i] = RL(0.0);
  if constexpr (L::kMtu > 0)
    for (int i = ln; i < L::kMtu; i += L::kLanes) E.act_bar[i] = RL(0.0);
  for (int i = ln; i < od; i += L::kLanes) E.obs[i] = A.obs_in[((size_t)A.h * A.N + env) * od + i];
  __syncthreads();
  obs_normalize<L::kLanes>(A, m, E.obs, ln);
  mlp_forward<L::kLanes>(A.critic, E.obs, E.h0, E.h1, E.y, E.xb16, ln, E.gb, E.lnst);
  // terminal value discounted from the start of the last segment (early termination)
  const int eh = m->term ? A.h - A.seg_ws[(size_t)A.h * A.N + env] : A.h;
  real c = -m_pow(A.gamma, (real)eh) * A.scale;
  if (ln == 0) E.y[0] = c;
  __syncthreads();
  mlp_vjp_input<L::kLanes>(A.critic, E.h0, E.h1, E.y, E.gb, E.obs, E.xb16, ln, E.lnst);
  obs_adjoint_scale<L::kLanes>(A, m, E.obs, ln);
  // E.obs now holds obs_bar; E.a holds a_prev of s_h
  task_obs_vjp<L::kLanes>(m, E.q, E.obs, E.qb, E.qdb, E.abar, E.act_bar, ln);
  if (A.grad_s_h) {
    const real* gs = A.grad_s_h + (size_t)env * ns;
    for (int i = ln; i < nq; i += L::kLanes) E.qb[i] += gs[i];
    for (int i = ln; i < nv; i += L::kLanes) E.qdb[i] += gs[nq + i];
    if (m->has_last_action)
      for (int i = ln; i < na; i += L::kLanes) E.abar[i] += gs[nq + nv + i];
    if constexpr (L::kMtu > 0) {
      const int o = nq + nv + (m->has_last_action ? na : 0);
      for (int i = ln; i < m->n_mtu; i += L::kLanes) E.act_bar[i] += gs[o + i];
    }
  }
  __syncthreads();
}

// frame-level reverse at frame t: E.qb/E.qdb hold the adjoint of the frame-start (q, qd)
// through the dynamics; E.abar holds dL/da_t except the reward term.  E.q/E.qd hold the
// frame-start state unless load_start (then it is read from the checkpoint arena).
template <class L>
__device__ __forceinline__ void adjoint_frame(const WinArgs& A, const Scal* __restrict__ m, L& E,
                                              int env, int t, int ln, bool load_start) {
  const int N = A.N, nq = m->nq, nv = m->nv, na = m->na, od = m->od, ns = m->ns, S = m->substeps;
  const int nck = m->nck;
  // frame-start state and a_t
  if (load_start) load_qqd(m, E, A.ckpt + ((size_t)(t * S / A.k) * N + env) * nck, ln);
  const real* at = A.actions_fw + ((size_t)t * N + env) * na;
  for (int i = ln; i < na; i += L::kLanes) E.a[i] = at[i];
  __syncthreads();
  const int et = m->term ? t - A.seg_ws[(size_t)t * N + env] : t;
  real c = -m_pow(A.gamma, (real)et) * A.scale;
  task_reward_vjp<L::kLanes>(m, E.q, E.qd, E.a, c, E.qb, E.qdb, E.abar, ln);
  real* da = A.dL_da + ((size_t)t * N + env) * na;
  for (int i = ln; i < na; i += L::kLanes) da[i] = E.abar[i];
  // a_prev of s_t is a_{t-1} (or the a_prev of s_0); its adjoint starts at zero
  __syncthreads();
  if (A.closed_loop) {
    // the actor's hidden activations as the forward stored them (the values a re-evaluation
    // on the stored observation would give, bit for bit)
    {
      const real* hs = A.hid + ((size_t)t * N + env) * A.hid_w;
      const int d1 = A.actor.nl > 1 ? A.actor.dims[1] : 0, d2 = A.actor.nl > 2 ? A.actor.dims[2] : 0;
      for (int i = ln; i < d1; i += L::kLanes) E.h0[i] = hs[i];
      for (int i = ln; i < d2; i += L::kLanes) E.h1[i] = hs[d1 + i];
      if (A.actor.ln && ln < 2 * (A.actor.nl - 1)) E.lnst[ln] = hs[d1 + d2 + ln];
    }
    __syncthreads();
    for (int i = ln; i < na; i += L::kLanes) E.y[i] = E.abar[i] * squash_grad(m, E.a[i]);
    __syncthreads();
    mlp_vjp_input<L::kLanes>(A.actor, E.h0, E.h1, E.y, E.gb, E.obs, E.xb16, ln, E.lnst);
    SIM_PHASE(E, PH_AF_MLP);
    for (int i = ln; i < L::kMaxA; i += L::kLanes) E.abar[i] = RL(0.0);
    __syncthreads();
    obs_adjoint_scale<L::kLanes>(A, m, E.obs, ln);
    task_obs_vjp<L::kLanes>(m, E.q, E.obs, E.qb, E.qdb, E.abar, E.act_bar, ln);
  } else {
    for (int i = ln; i < L::kMaxA; i += L::kLanes) E.abar[i] = RL(0.0);
    __syncthreads();
  }
  (void)ns;
  (void)od;
}

// The inputs of one checkpoint segment's state rebuild (factor cache), loaded into registers a
// segment ahead of their use: the checkpoint (lane ln: q[ln], qd[ln]) and the accelerations of
// the segment's first k - 1 substeps (lane ln: qdd[ln] of each).
struct FcSeg {
  real q, qd;
  real qdd[SIM_FC_MAXK - 1];
};
template <class L>
__device__ __forceinline__ void fc_seg_prefetch(const WinArgs& A, const Scal* __restrict__ m, FcSeg& G, int g, int env,
                                                int ln) {
  const int nq = m->nq, nv = m->nv, k = A.k, N = A.N;
  const real* ck = A.ckpt + ((size_t)g * N + env) * m->nck;
  G.q = (ln < nq) ? ck[ln] : RL(0.0);
  G.qd = (ln < nv) ? ck[nq + ln] : RL(0.0);
#pragma unroll
  for (int i = 0; i < SIM_FC_MAXK - 1; ++i)
    if (i < k - 1) G.qdd[i] = (ln < nv) ? A.fcq[(((size_t)g * k + i) * N + env) * nv + ln] : RL(0.0);
}
// the segment's pre-substep states from its checkpoint and cached accelerations: states 0 ..
// k - 2 into the per-env scratch pre, state k - 1 left in the block
template <class L>
__device__ __forceinline__ void fc_rebuild_states(const Scal* __restrict__ m, L& E, const JointRegs& jr, const FcSeg& G,
                                                  int k, real* __restrict__ pre, int ln) {
  if (ln < m->nq) E.q[ln] = G.q;
  if (ln < m->nv) E.qd[ln] = G.qd;
  wsync();
#pragma unroll
  for (int i = 0; i < SIM_FC_MAXK - 1; ++i) {
    if (i < k - 1) {
      store_qqd(m, E, pre + (size_t)i * m->nck, ln);
      fc_step_state(m, E, jr, G.qdd[i], ln);
    }
  }
}

// One environment's reverse window.  PATH: KP_TAPE, KP_FC, KP_CKPT (checkpoints without the
// factor cache) or KP_ANY.
template <int NV, class L, int PATH = KP_ANY>
__device__ __forceinline__ void window_adj_body(const WinArgs& A, int env, L& E) {
  const bool use_tape = PATH == KP_TAPE || (PATH == KP_ANY && A.tape_full);
  const bool use_fc = L::kMtu == 0 && (PATH == KP_FC || (PATH == KP_ANY && A.fc));
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int ln = grp_lane<L::kLanes>();
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nq = m->nq, nv = m->nv, na = m->na, ns = m->ns, N = A.N, k = A.k;
  const int nqv = m->nck;
  const TapeMap<L> TM = tape_map<L>(m, ln);
  const FcMap<L> FM = fc_map<L>(m, ln);
#ifdef SIM_PHASE_PROFILE
  phase_start<L::kLanes>(E.prof);
#endif
  adjoint_seed(A, m, E, env, ln);
  SIM_PHASE(E, PH_A_SEED);
  // E.abar holds the adjoint of a_prev(s_h) = a_{h-1}: it seeds dL/da_{h-1}
  Chol C;
  // factor cache: the next segment's rebuild inputs and the next entry, loaded ahead
  FcSeg NS;
  FcRegs<L> FP;
  if (use_fc) {
    const int G = A.h * S / k;
    fc_seg_prefetch<L>(A, m, NS, G - 1, env, ln);
    const size_t gi = (size_t)G * k - 1;
    fc_prefetch_entry(m, FM, FP, A.fc + (gi * N + env) * A.fc_ws, A.fcq + (gi * N + env) * nv, ln);
  }
  for (int t = A.h - 1; t >= 0; --t) {
    if (m->term && A.done_ws[(size_t)t * N + env]) {
      // frame t ended with a reset: s_{t+1} is a constant, nothing flows back through it
      for (int i = ln; i < L::kQ; i += L::kLanes) E.qb[i] = RL(0.0);
      for (int i = ln; i < L::kV; i += L::kLanes) E.qdb[i] = RL(0.0);
      for (int i = ln; i < L::kMaxA; i += L::kLanes) E.abar[i] = RL(0.0);
      if constexpr (L::kMtu > 0)
        for (int i = ln; i < L::kMtu; i += L::kLanes) E.act_bar[i] = RL(0.0);
      __syncthreads();
    }
    const real* at = A.actions_fw + ((size_t)t * N + env) * na;
    for (int i = ln; i < na; i += L::kLanes) E.a[i] = at[i];
    if (use_tape) {
      // the forward stored every substep's pre-state and linearisation; the next (earlier)
      // entry is loaded into registers while the current one is reversed
      TapeRegs<L> P;
      tape_prefetch<L>(TM, P, A.tape + (((size_t)t * S + S - 1) * N + env) * A.tape_ws, ln);
      for (int sub = S - 1; sub >= 0; --sub) {
        int fb;
        tape_load_regs<NV>(m, TM, E, C, fb, ln, P);
        if (sub > 0) tape_prefetch<L>(TM, P, A.tape + (((size_t)t * S + sub - 1) * N + env) * A.tape_ws, ln);
        SIM_PHASE(E, PH_TAPE_PREFETCH);
        if (fb) substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
        substep_adjoint_core<NV>(m, E, jr, cr, ln, C, fb);
      }
    } else if (use_fc) {
      // factor cache: per segment, the pre-substep states are rebuilt from the checkpoint with
      // the cached accelerations, then each substep is reversed from its state, its cached
      // factor and its recomputed kinematics; every load is issued a substep (entries) or a
      // segment (rebuild inputs) ahead of its use
      real* pre = A.tape + (size_t)env * k * nqv;
      for (int sg = S / k - 1; sg >= 0; --sg) {
        const int g = (t * S + sg * k) / k;
        const FcSeg CS = NS;
        if (g > 0) fc_seg_prefetch<L>(A, m, NS, g - 1, env, ln);
        fc_rebuild_states(m, E, jr, CS, k, pre, ln);
        FP.q = (ln < m->nq) ? E.q[ln] : RL(0.0);
        FP.qd = (ln < nv) ? E.qd[ln] : RL(0.0);
        SIM_PHASE(E, PH_FC_STATES);
        for (int i = k - 1; i >= 0; --i) {
          int fb;
          fc_load_regs(m, FM, E, fb, ln, FP);
          if (i > 0) {
            const size_t gi = (size_t)g * k + i - 1;
            fc_prefetch(m, FM, FP, A.fc + (gi * N + env) * A.fc_ws, A.fcq + (gi * N + env) * nv,
                        pre + (size_t)(i - 1) * nqv, ln);
          } else if (g > 0) {
            const size_t gi = (size_t)g * k - 1;
            fc_prefetch_entry(m, FM, FP, A.fc + (gi * N + env) * A.fc_ws, A.fcq + (gi * N + env) * nv, ln);
          }
          SIM_PHASE(E, PH_TAPE_PREFETCH);
          if (fb) {
            substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
          } else {
            // the factor enters registers only now: it is not live across the kinematics
            substep_kinematics(m, E, jr, cr, ln);
            int fb2;
            factor_from_block<NV>(m, E, C, fb2, ln);
            SIM_PHASE(E, PH_TAPE_LOAD);
          }
          substep_adjoint_core<NV>(m, E, jr, cr, ln, C, fb);
        }
      }
    } else {
      real* tseg = A.tape + (size_t)env * (k - 1) * A.tape_ws;
      for (int sg = S / k - 1; sg >= 0; --sg) {
        int c = (t * S + sg * k) / k;
        const real* ck = A.ckpt + ((size_t)c * N + env) * nqv;
        load_qqd(m, E, ck, ln);
        SIM_PHASE(E, PH_CKPT);
        // recompute the segment from its checkpoint, recording pre-states and
        // linearisations; the last substep's linearisation stays on chip
        for (int i = 0; i < k - 1; ++i) {
          int fb;
          substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
          tape_store<NV>(TM, E, C, fb, ln, tseg + (size_t)i * A.tape_ws);
          commit_substep(m, E, ln);
        }
        // the segment's recorded entries are loaded into registers one ahead of their use
        TapeRegs<L> P;
        {
          int fb;
          substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
          if (k >= 2) tape_prefetch<L>(TM, P, tseg + (size_t)(k - 2) * A.tape_ws, ln);
          SIM_PHASE(E, PH_TAPE_PREFETCH);
          substep_adjoint_core<NV>(m, E, jr, cr, ln, C, fb);
        }
        for (int i = k - 2; i >= 0; --i) {
          int fb;
          tape_load_regs<NV>(m, TM, E, C, fb, ln, P);
          if (i > 0) tape_prefetch<L>(TM, P, tseg + (size_t)(i - 1) * A.tape_ws, ln);
          SIM_PHASE(E, PH_TAPE_PREFETCH);
          if (fb) substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
          substep_adjoint_core<NV>(m, E, jr, cr, ln, C, fb);
        }
      }
    }
    // the reverse sweep ends on the frame's first substep: E.q/E.qd = s_t
    adjoint_frame(A, m, E, env, t, ln, false);
    SIM_PHASE(E, PH_A_FRAME);
  }
  real* d0 = A.dL_ds0 + (size_t)env * ns;
  for (int i = ln; i < nq; i += L::kLanes) d0[i] = E.qb[i];
  for (int i = ln; i < nv; i += L::kLanes) d0[nq + i] = E.qdb[i];
  if (m->has_last_action)
    for (int i = ln; i < na; i += L::kLanes) d0[nq + nv + i] = E.abar[i];
  if constexpr (L::kMtu > 0) {
    const int o = nq + nv + (m->has_last_action ? na : 0);
    for (int i = ln; i < m->n_mtu; i += L::kLanes) d0[o + i] = E.act_bar[i];
  }
#ifdef SIM_PHASE_PROFILE
  phase_flush<L::kLanes>(E.prof, A.prof);
#endif
}

// One workgroup of one wavefront runs 64 / L::kLanes environments, each on L::kLanes lanes
// with its own LDS block (full layouts: one environment per wavefront).
template <int NV, class L, int PATH>
__global__ __launch_bounds__(SIM_WAVE) void k_window_fwd(WinArgs A) {
  constexpr int EPW = SIM_WAVE / L::kLanes;
  __shared__ L E[EPW];
  const int g = EPW == 1 ? 0 : (int)threadIdx.x / L::kLanes;
  window_fwd_body<NV, L, PATH>(A, blockIdx.x * EPW + g, E[g]);
}

template <int NV, class L, int PATH>
__global__ __launch_bounds__(SIM_WAVE) void k_window_adj(WinArgs A) {
  constexpr int EPW = SIM_WAVE / L::kLanes;
  __shared__ L E[EPW];
  const int g = EPW == 1 ? 0 : (int)threadIdx.x / L::kLanes;
  window_adj_body<NV, L, PATH>(A, blockIdx.x * EPW + g, E[g]);
}

// ======================================================================= mixed-morphology group
// One launch over the envs of several models: block b runs the envs of block b - start[s] of
// the model in work-table slot s (slots ordered by decreasing per-env cost, so the longest
// windows are dispatched first).  Each slot's model runs the DOF-specialised body of its own
// kernel in its own LDS layout: torque models one env per wavefront in the full layout or
// 64 / lanes envs per wavefront in the compact layout, muscle models the muscle layout.  The
// block's LDS (dynamic) is the largest any member needs; each slot views it in its layout.
__device__ __forceinline__ int group_slot(const GroupArgs& G, int b) {
  int s = 0;
  for (int i = 1; i < G.n; ++i) s = (b >= G.start[i]) ? i : s;
  return s;
}

template <bool ADJ, int NV, class L>
__device__ __forceinline__ void group_body(const WinArgs& A, int env, L& E) {
  if (ADJ) window_adj_body<NV>(A, env, E);
  else window_fwd_body<NV>(A, env, E);
}

template <bool ADJ>
__device__ __forceinline__ void group_torque(const GroupArgs& G, int s, int env, EnvLDS& E) {
  switch (G.nv[s]) {
#define SIM_GROUP_T(n) case n: group_body<ADJ, n>(G.A[s], env, E); break;
    SIM_NV_LIST(SIM_GROUP_T)
#undef SIM_GROUP_T
    default: group_body<ADJ, SIM_MAXV>(G.A[s], env, E);
  }
}

template <bool ADJ>
__device__ __forceinline__ void group_muscle(const GroupArgs& G, int s, int env, EnvLDSM& E) {
  switch (G.nv[s]) {
#define SIM_GROUP_M(n) case n: group_body<ADJ, n>(G.A[s], env, E); break;
    SIM_NV_LIST_MTU(SIM_GROUP_M)
#undef SIM_GROUP_M
    default: group_body<ADJ, SIM_MAXV>(G.A[s], env, E);
  }
}

template <bool ADJ, int LN>
__device__ __forceinline__ void group_compact(const GroupArgs& G, int s, int blk, char* buf) {
  constexpr int EPW = SIM_WAVE / LN;
  EnvLDSC<LN>* E = reinterpret_cast<EnvLDSC<LN>*>(buf);
  const int g = EPW == 1 ? 0 : (int)threadIdx.x / LN;
  const int env = blk * EPW + g;
  switch (G.nv[s]) {
#define SIM_GROUP_C(n) case n: group_body<ADJ, n>(G.A[s], env, E[g]); break;
    SIM_NV_LIST_SMALL(SIM_GROUP_C)
#undef SIM_GROUP_C
    default: group_body<ADJ, SIM_CV>(G.A[s], env, E[g]);
  }
}

template <bool ADJ>
__global__ __launch_bounds__(SIM_WAVE) void k_group(GroupArgs G) {
  extern __shared__ __attribute__((aligned(16))) char gbuf[];
  const int s = group_slot(G, blockIdx.x);
  const int blk = blockIdx.x - G.start[s];
  if (G.mtu[s]) {
    group_muscle<ADJ>(G, s, blk, *reinterpret_cast<EnvLDSM*>(gbuf));
    return;
  }
  if constexpr (SIM_COMPACT) {
    if (G.lanes[s] == 16) { group_compact<ADJ, 16>(G, s, blk, gbuf); return; }
    if (G.lanes[s] == 32) { group_compact<ADJ, 32>(G, s, blk, gbuf); return; }
    if (G.lanes[s] == 64) { group_compact<ADJ, 64>(G, s, blk, gbuf); return; }
  }
  group_torque<ADJ>(G, s, blk, *reinterpret_cast<EnvLDS*>(gbuf));
}

#if SIM_EMIT_MAIN
// ======================================================================= plain path kernels
// One launch per frame start and one per substep; the state goes through HBM between
// launches (ckpt holds every substep's state, k = 1).
__global__ __launch_bounds__(SIM_WAVE) void k_plain_frame(WinArgs A, int t) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nqv = m->nq + m->nv, N = A.N, na = m->na;
  if (t == 0) {
    load_state(m, E, A.s0 + (size_t)env * m->ns, ln);
    store_qqd(m, E, A.ckpt + (size_t)env * nqv, ln);
    if (ln == 0 && A.fallback) A.fallback[env] = 0;
    if (ln == 0 && A.adhesive) A.adhesive[env] = 0;
  } else {
    load_qqd(m, E, A.ckpt + ((size_t)(t * S) * N + env) * nqv, ln);
    const real* ap = A.actions + ((size_t)(t - 1) * N + env) * na;
    for (int i = ln; i < na; i += SIM_WAVE) E.a[i] = ap[i];
    __syncthreads();
  }
  frame_begin(A, m, E, env, t, ln);
}

template <int NV>
__global__ __launch_bounds__(SIM_WAVE) void k_plain_substep(WinArgs A, int t, int sub) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nqv = m->nq + m->nv, N = A.N, na = m->na;
  int gi = t * S + sub;
  load_qqd(m, E, A.ckpt + ((size_t)gi * N + env) * nqv, ln);
  const real* at = A.actions + ((size_t)t * N + env) * na;
  for (int i = ln; i < na; i += SIM_WAVE) E.a[i] = at[i];
  __syncthreads();
  Chol C;
  int fb;
  substep_forward<NV>(m, E, jr, cr, ln, C, true, fb);
  store_qqd(m, E, A.ckpt + ((size_t)(gi + 1) * N + env) * nqv, ln);
  if (ln == 0 && A.fallback) A.fallback[env] += fb;
  if (ln == 0 && A.adhesive) A.adhesive[env] += E.nadh;
}

__global__ __launch_bounds__(SIM_WAVE) void k_plain_end(WinArgs A) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nqv = m->nq + m->nv, N = A.N, na = m->na;
  load_qqd(m, E, A.ckpt + ((size_t)(A.h * S) * N + env) * nqv, ln);
  const real* ap = A.actions + ((size_t)(A.h - 1) * N + env) * na;
  for (int i = ln; i < na; i += SIM_WAVE) E.a[i] = ap[i];
  __syncthreads();
  window_end(A, m, E, env, ln);
}

template <class L>
__device__ __forceinline__ void adj_load(const Scal* __restrict__ m, L& E, const real* src, int ln) {
  int nq = m->nq, nv = m->nv, na = m->na;
  for (int i = ln; i < SIM_MAXQ; i += SIM_WAVE) E.qb[i] = i < nq ? src[i] : RL(0.0);
  for (int i = ln; i < SIM_MAXV; i += SIM_WAVE) E.qdb[i] = i < nv ? src[nq + i] : RL(0.0);
  for (int i = ln; i < L::kMaxA; i += SIM_WAVE) E.abar[i] = i < na ? src[nq + nv + i] : RL(0.0);
  __syncthreads();
}
template <class L>
__device__ __forceinline__ void adj_store(const Scal* __restrict__ m, const L& E, real* dst, int ln) {
  int nq = m->nq, nv = m->nv, na = m->na;
  for (int i = ln; i < nq; i += SIM_WAVE) dst[i] = E.qb[i];
  for (int i = ln; i < nv; i += SIM_WAVE) dst[nq + i] = E.qdb[i];
  for (int i = ln; i < na; i += SIM_WAVE) dst[nq + nv + i] = E.abar[i];
}

__global__ __launch_bounds__(SIM_WAVE) void k_plain_adj_seed(WinArgs A) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  adjoint_seed(A, m, E, env, ln);
  adj_store(m, E, A.adj + (size_t)env * (m->nq + m->nv + m->na), ln);
}

template <int NV>
__global__ __launch_bounds__(SIM_WAVE) void k_plain_adj_substep(WinArgs A, int t, int sub) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int S = m->substeps, nqv = m->nq + m->nv, N = A.N, na = m->na;
  real* adj = A.adj + (size_t)env * (nqv + na);
  adj_load(m, E, adj, ln);
  load_qqd(m, E, A.ckpt + ((size_t)(t * S + sub) * N + env) * nqv, ln);
  const real* at = A.actions_fw + ((size_t)t * N + env) * na;
  for (int i = ln; i < na; i += SIM_WAVE) E.a[i] = at[i];
  __syncthreads();
  substep_adjoint<NV>(m, E, jr, cr, ln);
  adj_store(m, E, adj, ln);
}

__global__ __launch_bounds__(SIM_WAVE) void k_plain_adj_frame(WinArgs A, int t) {
  __shared__ EnvLDS E;
  const Scal scl = load_scal(A.model);
  const Scal* m = &scl;
  const int env = blockIdx.x, ln = threadIdx.x;
  JointRegs jr;
  ContactRegs cr;
  load_regs(A.model, E, ln, jr, cr);
  const int nqv = m->nq + m->nv, na = m->na, ns = m->ns, nq = m->nq, nv = m->nv;
  real* adj = A.adj + (size_t)env * (nqv + na);
  adj_load(m, E, adj, ln);
  adjoint_frame(A, m, E, env, t, ln, true);
  adj_store(m, E, adj, ln);
  if (t == 0) {
    real* d0 = A.dL_ds0 + (size_t)env * ns;
    for (int i = ln; i < nq; i += SIM_WAVE) d0[i] = E.qb[i];
    for (int i = ln; i < nv; i += SIM_WAVE) d0[nq + i] = E.qdb[i];
    if (m->has_last_action)
      for (int i = ln; i < na; i += SIM_WAVE) d0[nq + nv + i] = E.abar[i];
  }
}

// zero-padded weight copies: WT [in][pad64(out)] and Wp [out][pad64(in)] from W [out][in]
__global__ void k_prep_weights(const real* __restrict__ W, real* __restrict__ WT, real* __restrict__ Wp,
                               int no, int ni) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int nop = pad64(no), nip = pad64(ni);
  if (idx < ni * nop) {
    int i = idx / nop, o = idx % nop;
    WT[idx] = (o < no) ? W[(size_t)o * ni + i] : RL(0.0);
  }
  if (idx < no * nip) {
    int o = idx / nip, i = idx % nip;
    Wp[idx] = (i < ni) ? W[(size_t)o * ni + i] : RL(0.0);
  }
}

// BF16 operand tiles of one layer (see mlp_tiles_bf16): forward tiles of W and
// input-adjoint tiles of W^T, zero outside the matrix.
__global__ void k_prep_bf16(const real* __restrict__ W, uint16_t* __restrict__ Pf, uint16_t* __restrict__ Pb,
                            int no, int ni) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nf = (long)((no + 15) / 16) * ((ni + 31) / 32) * 512;
  const long nb = (long)((ni + 15) / 16) * ((no + 31) / 32) * 512;
  if (e < nf) {
    const int tile = (int)(e / 512), lane = (int)(e % 512) / 8, j = (int)(e % 8);
    const int nkt = (ni + 31) / 32;
    const int r = (tile / nkt) * 16 + lane % 16, k = (tile % nkt) * 32 + (lane / 16) * 8 + j;
    Pf[e] = (r < no && k < ni) ? f2bf((float)W[(size_t)r * ni + k]) : (uint16_t)0;
  }
  if (e < nb) {
    const int tile = (int)(e / 512), lane = (int)(e % 512) / 8, j = (int)(e % 8);
    const int nkt = (no + 31) / 32;
    const int r = (tile / nkt) * 16 + lane % 16, k = (tile % nkt) * 32 + (lane / 16) * 8 + j;
    Pb[e] = (r < ni && k < no) ? f2bf((float)W[(size_t)k * ni + r]) : (uint16_t)0;
  }
}

// ======================================================================= launchers
int launch_prep_bf16(const real* W, uint16_t* Pf, uint16_t* Pb, int n_out, int n_in, void* stream) {
  const long nf = (long)((n_out + 15) / 16) * ((n_in + 31) / 32) * 512;
  const long nb = (long)((n_in + 15) / 16) * ((n_out + 31) / 32) * 512;
  const long n = nf > nb ? nf : nb;
  hipLaunchKernelGGL(k_prep_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, W, Pf, Pb,
                     n_out, n_in);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prep_weights(const real* W, real* WT, real* Wp, int n_out, int n_in, void* stream) {
  int n = n_in * pad64(n_out) > n_out * pad64(n_in) ? n_in * pad64(n_out) : n_out * pad64(n_in);
  hipLaunchKernelGGL(k_prep_weights, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, W, WT, Wp, n_out, n_in);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The short-horizon actor loss of the window (Sec. 3.3, Eq. "policy_loss") from the frames'
// rewards and the terminal values: per env
//   l_e = -scale (sum_t gamma^(t - t0(t)) r_t + live_e gamma^(h - t0) V_e),
// with t0(t) the first frame of frame t's discount segment (0 without early termination) and
// live_e = 0 when the last frame ended in termination.  One block; the envs' losses are
// summed in a fixed order.
__global__ __launch_bounds__(1024) void k_window_loss(WinArgs A) {
  __shared__ real part[1024];
  const int N = A.N, h = A.h;
  const uint8_t* done = A.model->term ? A.done_ws : nullptr;
  real acc = RL(0.0);
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    real disc = RL(0.0);
    int t0 = 0;
    for (int t = 0; t < h; ++t) {
      disc += m_pow(A.gamma, (real)(t - t0)) * A.rewards[(size_t)t * N + e];
      if (done && done[(size_t)t * N + e]) t0 = t + 1;
    }
    const bool live = !(done && done[(size_t)(h - 1) * N + e]);
    const real le = -A.scale * (disc + (live ? m_pow(A.gamma, (real)(h - t0)) * A.value[e] : RL(0.0)));
    if (A.loss_env) A.loss_env[e] = le;
    acc += le;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && A.loss) A.loss[0] = part[0];
}

void launch_window_loss(const WinArgs& A, hipStream_t s) {
  if (A.loss_env || A.loss) hipLaunchKernelGGL(k_window_loss, dim3(1), dim3(1024), 0, s, A);
}
#endif  // SIM_EMIT_MAIN

// The full and muscle layouts have a kernel per launch form; the compact layouts (small
// models) one kernel that reads the form from its arguments.
template <int NV, class L>
static void launch_window(const WinArgs& A, int adjoint, hipStream_t s) {
  dim3 grid(A.N / (SIM_WAVE / L::kLanes)), block(SIM_WAVE);
  if constexpr (L::kLanes == SIM_WAVE) {
    if (adjoint) {
      if (A.tape_full) hipLaunchKernelGGL((k_window_adj<NV, L, KP_TAPE>), grid, block, 0, s, A);
      else if (L::kMtu == 0 && A.fc) hipLaunchKernelGGL((k_window_adj<NV, L, L::kMtu == 0 ? KP_FC : KP_CKPT>), grid, block, 0, s, A);
      else hipLaunchKernelGGL((k_window_adj<NV, L, KP_CKPT>), grid, block, 0, s, A);
    } else {
      if (A.tape_full) hipLaunchKernelGGL((k_window_fwd<NV, L, KP_TAPE>), grid, block, 0, s, A);
      else hipLaunchKernelGGL((k_window_fwd<NV, L, KP_CKPT>), grid, block, 0, s, A);
    }
  } else {
    if (adjoint) hipLaunchKernelGGL((k_window_adj<NV, L, KP_ANY>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_window_fwd<NV, L, KP_ANY>), grid, block, 0, s, A);
  }
}

#if SIM_EMIT_MAIN
template <int NV>
static void launch_plain(const WinArgs& A, int adjoint, int substeps, hipStream_t s) {
  dim3 grid(A.N), block(SIM_WAVE);
  if (!adjoint) {
    for (int t = 0; t < A.h; ++t) {
      hipLaunchKernelGGL(k_plain_frame, grid, block, 0, s, A, t);
      for (int sub = 0; sub < substeps; ++sub) hipLaunchKernelGGL(k_plain_substep<NV>, grid, block, 0, s, A, t, sub);
    }
    hipLaunchKernelGGL(k_plain_end, grid, block, 0, s, A);
  } else {
    hipLaunchKernelGGL(k_plain_adj_seed, grid, block, 0, s, A);
    for (int t = A.h - 1; t >= 0; --t) {
      for (int sub = substeps - 1; sub >= 0; --sub)
        hipLaunchKernelGGL(k_plain_adj_substep<NV>, grid, block, 0, s, A, t, sub);
      hipLaunchKernelGGL(k_plain_adj_frame, grid, block, 0, s, A, t);
    }
  }
}

template <int NV>
static void launch_torque_nv(const WinArgs& A, int adjoint, int plain, int substeps, int lanes, hipStream_t s) {
  if (plain) launch_plain<NV>(A, adjoint, substeps, s);
  else launch_window<NV, EnvLDS>(A, adjoint, s);
  (void)lanes;
}

#if !SIM_COMPACT
int launch_compact(const WinArgs&, int, int, int, void*) { return -1; }
#endif

// Torque-driven models have a kernel per DOF count in SIM_NV_LIST, muscle-driven ones per
// DOF count in SIM_NV_LIST_MTU, small models in the compact layout (lanes 16 / 32 / 64) per
// DOF count in SIM_NV_LIST_SMALL; every other model runs the padded kernel of its layout.  The
// plain path exists for torque-driven models in the full layout only (the host rejects the
// other cases).
static void launch_dispatch(const WinArgs& A, int adjoint, int plain, int substeps, int nv, int mtu, int lanes,
                            hipStream_t s) {
  if (mtu) {
    switch (nv) {
#define SIM_CASE_M(n) case n: launch_window<n, EnvLDSM>(A, adjoint, s); break;
      SIM_NV_LIST_MTU(SIM_CASE_M)
#undef SIM_CASE_M
      default: launch_window<SIM_MAXV, EnvLDSM>(A, adjoint, s);
    }
  } else if (lanes) {
    launch_compact(A, adjoint, nv, lanes, s);
  } else {
    switch (nv) {
#define SIM_CASE_T(n) case n: launch_torque_nv<n>(A, adjoint, plain, substeps, 0, s); break;
      SIM_NV_LIST(SIM_CASE_T)
#undef SIM_CASE_T
      default: launch_torque_nv<SIM_MAXV>(A, adjoint, plain, substeps, 0, s);
    }
  }
}

int launch_forward(const WinArgs& A, int plain, int substeps, int nv, int mtu, int lanes, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  launch_dispatch(A, 0, plain, substeps, nv, mtu, lanes, s);
  launch_window_loss(A, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint(const WinArgs& A, int plain, int substeps, int nv, int mtu, int lanes, void* stream) {
  launch_dispatch(A, 1, plain, substeps, nv, mtu, lanes, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#endif  // SIM_EMIT_MAIN

#if SIM_EMIT_COMPACT
template <int NV>
static void launch_compact_nv(const WinArgs& A, int adjoint, int lanes, hipStream_t s) {
  if (lanes == 16) launch_window<NV, EnvLDSC<16>>(A, adjoint, s);
  else if (lanes == 32) launch_window<NV, EnvLDSC<32>>(A, adjoint, s);
  else launch_window<NV, EnvLDSC<64>>(A, adjoint, s);
}

int launch_compact(const WinArgs& A, int adjoint, int nv, int lanes, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (nv) {
#define SIM_CASE_C(n) case n: launch_compact_nv<n>(A, adjoint, lanes, s); break;
    SIM_NV_LIST_SMALL(SIM_CASE_C)
#undef SIM_CASE_C
    default: launch_compact_nv<SIM_CV>(A, adjoint, lanes, s);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
#endif  // SIM_EMIT_COMPACT

#if SIM_EMIT_MAIN
// LDS bytes of one group block for a member: muscle layout, full torque layout (lanes 0) or
// 64 / lanes compact layouts
size_t group_lds_bytes(int lanes, int mtu) {
  if (mtu) return sizeof(EnvLDSM);
  if (!SIM_COMPACT) return sizeof(EnvLDS);
  if (lanes == 16) return 4 * sizeof(EnvLDSC<16>);
  if (lanes == 32) return 2 * sizeof(EnvLDSC<32>);
  if (lanes == 64) return sizeof(EnvLDSC<64>);
  return sizeof(EnvLDS);
}

int launch_group(const GroupArgs& G, int adjoint, int mtu, size_t lds_bytes, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  (void)mtu;
  int bad = adjoint ? launch_group_adj(G, lds_bytes, st) : launch_group_fwd(G, lds_bytes, st);
  if (!adjoint)
    for (int s = 0; s < G.n; ++s) launch_window_loss(G.A[s], st);
  return (bad || hipGetLastError() != hipSuccess) ? -1 : 0;
}

// the largest dynamic LDS the group kernels may be launched with (above the default limit
// of 64 KB the kernels must be allowed it once, before any launch or capture)
int prepare_group(size_t lds_bytes) {
  if (lds_bytes <= 65536) return 0;
  return (prepare_group_fwd(lds_bytes) || prepare_group_adj(lds_bytes)) ? -1 : 0;
}
#endif  // SIM_EMIT_MAIN

#if SIM_EMIT_GROUP_FWD
int launch_group_fwd(const GroupArgs& G, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_group<false>, dim3(G.start[G.n]), dim3(SIM_WAVE), lds_bytes, s, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int prepare_group_fwd(size_t lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group<false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) == hipSuccess ? 0 : -1;
}
#endif  // SIM_EMIT_GROUP_FWD

#if SIM_EMIT_GROUP_ADJ
int launch_group_adj(const GroupArgs& G, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_group<true>, dim3(G.start[G.n]), dim3(SIM_WAVE), lds_bytes, s, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int prepare_group_adj(size_t lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group<true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) == hipSuccess ? 0 : -1;
}
#endif  // SIM_EMIT_GROUP_ADJ
