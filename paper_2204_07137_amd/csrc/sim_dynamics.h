// One substep of the articulated-body dynamics and its adjoint, for one environment
// per wavefront.
//
// Forward (Sec. 3.1, Eq. "fwd_dynamics"): forward kinematics and velocities by pointer
// jumping over the tree's parent links, penalty contact and friction (Sec. 3.1 contact equation), joint limit
// penalty (Sec. 3.1 limit equation), RNEA bias b(q, qd) with gravity and contact
// wrenches, CRBA mass matrix, dense Cholesky M = L L^T, qdd = M^{-1}(tau - b) and a
// semi-implicit Euler step.
//
// Adjoint (Sec. 3.1, Eq. "backward"): the integrator is reversed explicitly; the
// solve is reversed with the cached factor (lambda = M^{-1} qdd_bar, the reuse of the
// factorisation that Sec. 3.1 describes); the dependence of qdd on (q, qd, a) is taken
// from the implicit function theorem on ID(q, qd, qdd, a) = M qdd + b - tau = 0, so that
// x_bar -= d/dx [lambda^T ID] at the solved qdd.  That scalar is sum_b w_b . f_b^net
// (w_b = virtual body velocities of lambda, f_b^net = Newton-Euler force minus contact
// wrench) minus the limit and actuation work; its derivatives are evaluated in closed
// form from subtree sums of spatial vectors (no derivative of M or of the factor).

#define SIM_PAIR_ROUNDS (SIM_MAXPAIR / SIM_WAVE)
// per-lane joint constants kept in registers; the larger per-joint tables (offsets, axes,
// centres of mass, inertias, mass-matrix pairs) are copied to LDS once per kernel
struct JointRegs {
  int par, type, qa, va, depth, act, lim, npair;
  unsigned int cmask;
  real lo, hi, gear, mass, arm;
};
struct ContactRegs {
  int body;
  f3 pos;
  real rad;
};

// Muscle accumulators: a table of SIM_MAXJ x 6 values padded to an odd stride (so the copies
// of one entry sit in different banks); the forward keeps SIM_MUS_CF copies of the wrench
// table, the adjoint SIM_MUS_CA copies of each of its three tables.
#define SIM_MUS_STRIDE (SIM_MAXJ * 6 + 1)
#define SIM_MUS_CF 11
#define SIM_MUS_CA 3
static_assert(3 * SIM_MUS_CA <= SIM_MUS_CF, "adjoint muscle tables fit the forward's space");

// Per-environment LDS of one environment.  MAXA: action capacity; NMTU: muscle capacity
// (0 for torque-driven models, whose layout then carries no muscle fields); LANES: the lanes
// of a wavefront that simulate the environment (64, or 16 / 32 with 64 / LANES environments
// per wavefront); CJ, CV, CC, COBS, CHID, CPAIR: capacities of frames, DOFs, contact spheres,
// observation, MLP width and mass-matrix pairs.
template <int MAXA, int NMTU, int LANES = SIM_WAVE, int CJ = SIM_MAXJ, int CV = SIM_MAXV, int CC = SIM_MAXC,
          int COBS = SIM_MAXOBS, int CHID = SIM_MAXHID, int CPAIR = SIM_MAXPAIR>
struct EnvLDST {
  static constexpr int kMtu = NMTU;
  static constexpr int kMaxA = MAXA;
  static constexpr int kLanes = LANES;
  static constexpr int kJ = CJ, kV = CV, kQ = CV + 1, kC = CC, kObs = COBS, kHid = CHID, kPair = CPAIR;
  // the most 16-byte chunks a packed tape entry / a factor-cache entry of this layout can need,
  // per lane
  static constexpr int kTapeChunksPerLane = (sim_tape_chunk_cap(CJ, CV, CC, NMTU, (int)sizeof(real)) + LANES - 1) / LANES;
  static constexpr int kFcChunksPerLane = (sim_fc_chunk_cap(CV, (int)sizeof(real)) + LANES - 1) / LANES;
  // The linearisation of the current substep, one contiguous block whose fields
  // sim_tape_layout describes; a tape entry holds the words of it that the model uses
  // (for torque-driven models no R and p: those are rebuilt by any recomputation and never
  // read by the adjoint).
  struct __attribute__((aligned(16))) {
    real q[CV + 1], qd[CV];   // state before the substep
    real S[CJ][6], v[CJ][6], ab[CJ][6], Ib[CJ][10];
    real cf[CC][3], cx[CC][3], cvel[CC][3], cdep[CC];
    real qdd[CV], qdn[CV];
    real M[CV][CV + 1];    // mass matrix, then the Cholesky rows
    real tdinv[CV], tfb[CV];
    real R[CJ][9], p[CJ][3];
    real act[NMTU];                    // muscle activations before the substep
  };
  real a[MAXA];
  real qn[CV + 1];
  real actn[NMTU];                     // activations after the substep
  real act_bar[NMTU];
  // substep scratch: the forward's Newton-Euler forces, CRBA columns and composite
  // inertias, and the adjoint's per-body terms with their subtree sums (never live together)
  union {
    struct {
      real F[CJ][6], Fi[CJ][6];
      real Ic[CJ][10];
    };
    real acc[CJ][42];
  };
  real vec[CV];
  real O[4];
  // adjoint
  real W[CJ][6], A[CJ][6];
  real cAb[CC][6], cVb[CC][6];
  real qb[CV + 1], qdb[CV], abar[MAXA];
  real lam[CV], dPq[CV], dPqd[CV];
  // topology copies for arbitrary-index lookups
  int t_next_sib[CJ], t_type[CJ], t_va[CJ], t_parent[CJ], t_qa[CJ];
  unsigned short t_ts[4][SIM_MAXTS] __attribute__((aligned(16)));   // subtree-sum schedule
  real arm[CV];
  real j_off[CJ][3], j_ax[CJ][3], j_com[CJ][3], j_I6[CJ][6];
  int pairs[CPAIR];
  int nadh;   // contacts of the last substep whose normal force pulled (see the contact phase)
  // policy / critic
  real obs[COBS];
  union {
    struct {
      real h0[CHID], h1[CHID], y[CHID], gb[CHID];
      uint16_t xb16[CHID] __attribute__((aligned(16)));   // BF16 layer operand
    };
    double M64[CV][CV];   // FP64 refactorisation (never live at the same time as the MLP)
    // per-body muscle wrenches and their adjoint terms (substep-local), accumulated in
    // several copies (see muscle_wrenches); copy 0 of each table holds the sums
    real mus[NMTU > 0 ? SIM_MUS_CF * SIM_MUS_STRIDE : 1];
  };
  real red[4];
  real lnst[2 * SIM_MAXL];   // per hidden layer: mean and inverse deviation of its normalisation
#ifdef SIM_PHASE_PROFILE
  unsigned long long prof[SIM_NPHASE + 1];   // phase cycle totals and the last mark's time
#endif
};
typedef EnvLDST<SIM_MAXA, 0> EnvLDS;             // torque-driven models
typedef EnvLDST<SIM_MAXAM, SIM_MAXMTU> EnvLDSM;  // muscle-driven models
// small torque-driven models: LN lanes per environment, 64 / LN environments per wavefront
template <int LN>
using EnvLDSC = EnvLDST<SIM_CA, 0, LN, SIM_CJ, SIM_CV, SIM_CC, SIM_COBS, SIM_CHID, SIM_CPAIR>;
// four environments per CU (160 KB of LDS) in FP32, for both layouts
static_assert(sizeof(real) != 4 || sizeof(EnvLDSM) <= 40960, "muscle LDS layout exceeds a quarter of the CU's LDS");

template <class L>
__device__ __forceinline__ void load_regs(const DevModel* __restrict__ m, L& E, int ln,
                                          JointRegs& jr, ContactRegs& cr) {
  constexpr int LN = L::kLanes;
  int j = ln < m->J ? ln : 0;
  jr.par = m->parent[j]; jr.type = m->jtype[j]; jr.qa = m->qadr[j]; jr.va = m->vadr[j];
  jr.depth = ln < m->J ? m->depth[j] : -1;
  jr.act = m->act_of_joint[j]; jr.lim = m->limited[j];
  jr.lo = m->lower[j]; jr.hi = m->upper[j]; jr.gear = m->gear[j]; jr.mass = m->mass[j];
  jr.cmask = ln < m->J ? m->cmask[j] : 0u;
  jr.arm = m->armature[m->vadr[j]];
  jr.npair = m->npair;
  for (int p = ln; p < m->npair; p += LN) E.pairs[p] = m->pair[p];
  for (int i = ln; i < 2 * SIM_MAXTS; i += LN)
    reinterpret_cast<unsigned int*>(&E.t_ts[0][0])[i] = reinterpret_cast<const unsigned int*>(&m->ts_edge[0][0])[i];
  for (int f = ln; f < L::kJ; f += LN) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      E.j_off[f][k] = m->offset[3 * f + k];
      E.j_ax[f][k] = m->axis[3 * f + k];
      E.j_com[f][k] = m->com[3 * f + k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) E.j_I6[f][k] = m->inertia[6 * f + k];
  }
  int c = ln < m->nc ? ln : 0;
  cr.body = m->cbody[c]; cr.pos = ld3(&m->cpos[3 * c]); cr.rad = m->crad[c];
  for (int f = ln; f < L::kJ; f += LN) {
    E.t_next_sib[f] = m->next_sib[f]; E.t_type[f] = m->jtype[f];
    E.t_va[f] = m->vadr[f]; E.t_parent[f] = m->parent[f]; E.t_qa[f] = m->qadr[f];
  }
  for (int f = ln; f < L::kV; f += LN) E.arm[f] = m->armature[f];
  wsync();
}

// --------------------------------------------------------------- contact law
// Normal f_n = (-kn + kd ddot) min(d, 0) (active for d < 0), friction only while d < 0:
// viscous -kt v_t when kt |v_t| <= mu |f_n| (ties included), else -mu |f_n| v_t / |v_t|.
// Returns the world force and, if wanted, df/dd (3) and df/dv (3x3 row-major).
__device__ __forceinline__ f3 contact_force(const Scal* __restrict__ m, real d, f3 v,
                                            bool want_d, f3* dfdd, real* dfdv) {
  f3 f = mk3(RL(0.0), RL(0.0), RL(0.0));
  if (want_d) {
    *dfdd = mk3(RL(0.0), RL(0.0), RL(0.0));
#pragma unroll
    for (int k = 0; k < 9; ++k) dfdv[k] = RL(0.0);
  }
  if (!(d < RL(0.0))) return f;
  real kn = m->kn, kd = m->kd, kt = m->kt, mu = m->mu;
  real stiff = -kn + kd * v.z;
  real fn = stiff * d;
  real vt2 = v.x * v.x + v.y * v.y;
  real afn = m_fabs(fn);
  real lim = mu * afn;
  f.z = fn;
  bool viscous = kt * kt * vt2 <= lim * lim;
  if (viscous) {
    f.x = -kt * v.x;
    f.y = -kt * v.y;
  } else {
    real vn = m_sqrt(vt2);
    real s = lim / vn;
    f.x = -s * v.x;
    f.y = -s * v.y;
  }
  if (want_d) {
    // d fn / d d = stiff, d fn / d vz = kd d
    dfdd->z = stiff;
    dfdv[8] = kd * d;
    if (viscous) {
      dfdv[0] = -kt;
      dfdv[4] = -kt;
    } else {
      real vn = m_sqrt(vt2);
      real tx = v.x / vn, ty = v.y / vn;
      real sg = fn > RL(0.0) ? RL(1.0) : (fn < RL(0.0) ? -RL(1.0) : RL(0.0));
      real dft_dfn_x = -mu * sg * tx, dft_dfn_y = -mu * sg * ty;
      dfdd->x = dft_dfn_x * stiff;
      dfdd->y = dft_dfn_y * stiff;
      dfdv[2] = dft_dfn_x * kd * d;
      dfdv[5] = dft_dfn_y * kd * d;
      real c = -lim / vn;
      dfdv[0] = c * (RL(1.0) - tx * tx);
      dfdv[1] = c * (-tx * ty);
      dfdv[3] = c * (-ty * tx);
      dfdv[4] = c * (RL(1.0) - ty * ty);
    }
  }
  return f;
}

// rotation matrix of the normalised quaternion (w, x, y, z)
__device__ __forceinline__ void quat_rot(real w, real x, real y, real z, real* R) {
  real n2 = w * w + x * x + y * y + z * z;
  real s = RL(2.0) / n2;
  R[0] = RL(1.0) - s * (y * y + z * z); R[1] = s * (x * y - w * z);       R[2] = s * (x * z + w * y);
  R[3] = s * (x * y + w * z);       R[4] = RL(1.0) - s * (x * x + z * z); R[5] = s * (y * z - w * x);
  R[6] = s * (x * z - w * y);       R[7] = s * (y * z + w * x);       R[8] = RL(1.0) - s * (x * x + y * y);
}

// coefficients of the half-angle exponential exp((dt/2) w): c(u), s(u) with u = |w|^2,
// and their derivatives in u
__device__ __forceinline__ void dq_coeffs(real u, real hh, real& c, real& s, real& dc, real& ds) {
  real x2 = u * hh * hh;
  if (x2 < RL(1e-2)) {
    c = RL(1.0) - x2 * (RL(0.5) - x2 * (RL(1.0) / RL(24.0) - x2 * (RL(1.0) / RL(720.0))));
    s = hh * (RL(1.0) - x2 * (RL(1.0) / RL(6.0) - x2 * (RL(1.0) / RL(120.0) - x2 * (RL(1.0) / RL(5040.0)))));
    ds = hh * hh * hh * (-RL(1.0) / RL(6.0) + x2 * (RL(2.0) / RL(120.0) - x2 * (RL(3.0) / RL(5040.0))));
  } else {
    real n = m_sqrt(u);
    real sn, cs;
    m_sincos(n * hh, &sn, &cs);
    c = cs;
    s = sn / n;
    ds = (hh * c - s) / (RL(2.0) * u);
  }
  dc = -RL(0.5) * hh * s;
}

// --------------------------------------------------------------- dense Cholesky (row per lane)
// The factor of one environment lives in the registers of its wavefront: lane i holds row i
// (row[k] = L[i][k], k <= i) and column i (col[k] = L[k][i], k >= i); dinv[k] = 1 / L[k][k]
// is held by every lane.  NV is the compile-time DOF count: rows beyond the model's nv are
// padded with the identity, which leaves the factor and the solution of the real block
// unchanged, so no per-step guards are needed.
struct Chol {
  real row[SIM_MAXV], col[SIM_MAXV], dinv[SIM_MAXV];
};

// On entry C.row[k] = M[ln][k].  Right-looking factorisation; the column-k entries of the
// other rows are broadcast with readlane.
template <int NV, int LN>
__device__ __forceinline__ void chol_factor(Chol& C, int ln, real& minpiv) {
  minpiv = RL(3.0e38);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    real piv = bcast<LN>(C.row[k], k);
    minpiv = m_fmin(minpiv, piv);
    real inv = m_rsqrt(piv);
    real d = piv * inv;
    C.dinv[k] = inv;
    real lk = (ln == k) ? d : C.row[k] * inv;
    C.row[k] = lk;
    real ljk[NV];
#pragma unroll
    for (int j = k + 1; j < NV; ++j) ljk[j] = bcast<LN>(lk, j);
#pragma unroll
    for (int j = k + 1; j < NV; ++j) C.row[j] = m_fma(-lk, ljk[j], C.row[j]);
  }
}

// solve L L^T x = b for b given in lane ln (row ln)
template <int NV, int LN>
__device__ __forceinline__ real chol_solve(const Chol& C, int ln, real b) {
  real y = b;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    real yk = bcast<LN>(y, k) * C.dinv[k];
    y = (ln == k) ? yk : (ln > k ? m_fma(-C.row[k], yk, y) : y);
  }
#pragma unroll
  for (int k = NV - 1; k >= 0; --k) {
    real xk = bcast<LN>(y, k) * C.dinv[k];
    y = (ln == k) ? xk : (ln < k ? m_fma(-C.col[k], xk, y) : y);
  }
  return y;
}

// --------------------------------------------------------------- FP64 fallback factorisation
// When the FP32 factorisation meets a pivot below chol_thr times the largest diagonal (or
// a non-finite pivot), the environment's mass matrix is refactorised in double precision
// in LDS (lane = row) and both solves of the substep use that factor.
template <int NV, class L>
__device__ __forceinline__ void chol64_factor(L& E, int nv, int ln) {
  if (ln < NV) {
#pragma unroll 1
    for (int k = 0; k < NV; ++k)
      E.M64[ln][k] = (ln < nv && k < nv) ? (double)E.M[ln][k] : (ln == k ? 1.0 : 0.0);
  }
  wsync();
#pragma unroll 1
  for (int k = 0; k < NV; ++k) {
    double piv = E.M64[k][k];
    double d = sqrt(piv);
    double lk = (ln > k && ln < NV) ? E.M64[ln][k] / d : 0.0;
    wsync();
    if (ln == k) E.M64[k][k] = d;
    if (ln > k && ln < NV) E.M64[ln][k] = lk;
    wsync();
    if (ln > k && ln < NV)
#pragma unroll 1
      for (int j = k + 1; j <= ln; ++j) E.M64[ln][j] -= lk * E.M64[j][k];
    wsync();
  }
}

template <int NV, class L>
__device__ __forceinline__ double chol64_solve(L& E, int ln, double b) {
  constexpr int LN = L::kLanes;
  double y = b;
#pragma unroll 1
  for (int k = 0; k < NV; ++k) {
    double yk = bcast<LN>(y, k) / E.M64[k][k];
    if (ln == k) y = yk;
    else if (ln > k && ln < NV) y -= E.M64[ln][k] * yk;
  }
#pragma unroll 1
  for (int k = NV - 1; k >= 0; --k) {
    double xk = bcast<LN>(y, k) / E.M64[k][k];
    if (ln == k) y = xk;
    else if (ln < k) y -= E.M64[k][ln] * xk;
  }
  return y;
}

// --------------------------------------------------------------- subtree sums
// Adds every frame's row of a table into its parent's row, children before parents
// (frames are listed parents first); each active lane owns one column.  The parent index
// is broadcast from the lane that holds it; the LDS executes one wavefront's accesses in
// order, so a parent updated by an earlier edge is read back correctly without a wait.
__device__ __forceinline__ void tree_sum_cols(real* col, int stride, bool active, int J, int par_reg) {
  for (int j = J - 1; j >= 1; --j) {
    int p = __builtin_amdgcn_readlane(par_reg, j);
    if (active && p >= 0) col[p * stride] += col[j * stride];
  }
}

// The forward's subtree sums of 16 columns (Newton-Euler forces, composite inertias) along
// the model's schedule: lane = (group g of four, column c of 16); at each step every group
// adds one frame's row into its parent's.  A step holds no edge into a frame whose own
// incoming edges are not all done, and no two edges into one parent, so the groups touch
// disjoint rows and the LDS performs each step's accesses after the previous step's.
// With fewer than 64 lanes per environment a lane serves several groups, one after the
// other within each step (the groups of a step touch disjoint rows, so the order of a step's
// groups does not change any sum).
template <class L>
__device__ __forceinline__ void tree_sum_sched16(L& E, int nsteps, int ln) {
  constexpr int LN = L::kLanes, NG = SIM_WAVE / LN;   // schedule groups per lane
  const int c = ln & 15;
  real* col = (c < 6) ? &E.F[0][c] : &E.Ic[0][c - 6];
  const int st = (c < 6) ? 6 : 10;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  unsigned int w32[NG][SIM_MAXTS / 2];
#pragma unroll
  for (int r = 0; r < NG; ++r) {
    const int g = r * (LN / 16) + (ln >> 4);
    const u32x4* tp = reinterpret_cast<const u32x4*>(&E.t_ts[g][0]);
#pragma unroll
    for (int i = 0; i < SIM_MAXTS / 8; ++i) {
      const u32x4 v = tp[i];
      w32[r][4 * i] = v.x; w32[r][4 * i + 1] = v.y; w32[r][4 * i + 2] = v.z; w32[r][4 * i + 3] = v.w;
    }
  }
#pragma unroll
  for (int s = 0; s < SIM_MAXTS; ++s) {
    if (s < nsteps) {
#pragma unroll
      for (int r = 0; r < NG; ++r) {
        const unsigned int w = (w32[r][s >> 1] >> (16 * (s & 1))) & 0xffffu;
        if (w) {
          const int j = (int)(w & 31u), p = (int)((w >> 5) & 31u);
          col[p * st] += col[j * st];
        }
      }
    }
  }
}

// Sums of two spatial vectors over each frame's root path by pointer jumping: a round adds
// the partial sums of the frame the link names and takes over its link (ceil(log2(depth +
// 1)) rounds).  Values move between lanes by wavefront permutes, so every lane must be
// active.
template <int LN>
__device__ __forceinline__ sv pull_sv(sv x, int src) {
  return mksv(mk3(pull_g<LN>(x.a.x, src), pull_g<LN>(x.a.y, src), pull_g<LN>(x.a.z, src)),
              mk3(pull_g<LN>(x.l.x, src), pull_g<LN>(x.l.y, src), pull_g<LN>(x.l.z, src)));
}
template <int LN>
__device__ __forceinline__ void path_sum2(sv& x, sv& z, int link, int rounds) {
  for (int r = 0; r < rounds; ++r) {
    const int src = link >= 0 ? link : grp_lane<LN>();
    const sv yx = pull_sv<LN>(x, src);
    const sv yz = pull_sv<LN>(z, src);
    const int nl = pull_g<LN>(link, src);
    if (link >= 0) {
      x = addsv(yx, x);
      z = addsv(yz, z);
      link = nl;
    }
  }
}

// --------------------------------------------------------------- forward substep
// Uses E.q, E.qd, E.a.  Writes all intermediates to E and the new state to E.qn/E.qdn
// (and back to E.q/E.qd when inplace).  Lrow/Lcol keep the Cholesky factor.
// --------------------------------------------------------------- muscle-tendon units
// Unit i's path: points x_k (relative to O) fixed in body frames, segments u_k (unit) of
// length l_k, L = sum l_k, Ldot = sum u_k . (v_{k+1} - v_k).  Rigid tendon l_m = L - l_slack;
// tension F = max(0, F_max act f_l f_v) with f_l = exp(-((l_m/l_opt - 1)/w)^2) and
// f_v = 1 + Ldot/(v_max l_opt); point k receives F (u_k - u_{k-1}) (u_{-1} = u_{n-1} = 0).
struct MtuPath {
  f3 x[SIM_MAXMPT], v[SIM_MAXMPT], u[SIM_MAXMPT - 1];
  real il[SIM_MAXMPT - 1];   // 1 / segment length
  int b[SIM_MAXMPT];
  int np;
  real F, Fr, fl, fv, lt, L, Ld;
  real fmax, lopt;
};

template <class L>
__device__ __forceinline__ void mtu_path(const Scal* __restrict__ m, const L& E, int i, MtuPath& P,
                                         real act) {
  typedef real rv4 __attribute__((ext_vector_type(4)));
  const DevModel* __restrict__ T = m->tab;
  const rv4 par = *reinterpret_cast<const rv4*>(&T->mtu_par[4 * i]);
  P.np = (int)par[3];
  P.fmax = par[0];
  P.lopt = par[1];
#pragma unroll
  for (int k = 0; k < SIM_MAXMPT; ++k) {
    // the model tables repeat the last point in the slots past it
    const rv4 w = *reinterpret_cast<const rv4*>(&T->mtu_pt[4 * (k * SIM_MAXMTU + i)]);
    const int b = (int)w[3];
    f3 r = mk3(w[0], w[1], w[2]);
    P.b[k] = b;
    P.x[k] = add3(ld3(E.p[b]), mv3(E.R[b], r));
    P.v[k] = ptv(ldsv(E.v[b]), P.x[k]);
  }
  real Lp = RL(0.0), Ld = RL(0.0);
#pragma unroll
  for (int k = 0; k < SIM_MAXMPT - 1; ++k) {
    if (k + 1 < P.np) {
      f3 d = sub3(P.x[k + 1], P.x[k]);
      real l = m_sqrt(dot3(d, d));
      real il = RL(1.0) / l;
      P.u[k] = scl3(d, il);
      P.il[k] = il;
      Lp += l;
      Ld += dot3(P.u[k], sub3(P.v[k + 1], P.v[k]));
    } else {
      P.u[k] = mk3(RL(0.0), RL(0.0), RL(0.0));
      P.il[k] = RL(0.0);
    }
  }
  const real lopt = P.lopt;
  P.L = Lp;
  P.Ld = Ld;
  P.lt = (Lp - par[2]) / lopt;
  const real z = (P.lt - RL(1.0)) / m->fl_w;
  P.fl = m_exp(-z * z);
  P.fv = RL(1.0) + Ld / (m->vmax * lopt);
  P.Fr = P.fmax * act * P.fl * P.fv;
  P.F = P.Fr > RL(0.0) ? P.Fr : RL(0.0);
}

__device__ __forceinline__ f3 mtu_udiff(const MtuPath& P, int k) {
  f3 uf = (k < SIM_MAXMPT - 1) ? P.u[k] : mk3(RL(0.0), RL(0.0), RL(0.0));
  f3 ub = (k > 0) ? P.u[k - 1] : mk3(RL(0.0), RL(0.0), RL(0.0));
  return sub3(uf, ub);
}

__device__ __forceinline__ void lds_add6(real* dst, sv w) {
  atomicAdd(dst + 0, w.a.x); atomicAdd(dst + 1, w.a.y); atomicAdd(dst + 2, w.a.z);
  atomicAdd(dst + 3, w.l.x); atomicAdd(dst + 4, w.l.y); atomicAdd(dst + 5, w.l.z);
}

// Per-body wrench of all muscle tensions (about O), left in copy 0 of the wrench table
// (mus_fm).  One lane per unit.  Many units share a body, and LDS atomics to one address
// are serialised, so lane l adds into copy l % SIM_MUS_CF and the copies are summed
// afterwards in copy order; an instruction's additions to one address are performed in
// lane order, so the sums are reproducible.
template <class L>
__device__ __forceinline__ real* mus_fm(L& E, int b) { return &E.mus[b * 6]; }
template <class L>
__device__ __forceinline__ real* mus_ab(L& E, int b) { return &E.mus[SIM_MUS_CA * SIM_MUS_STRIDE + b * 6]; }
template <class L>
__device__ __forceinline__ real* mus_vb(L& E, int b) { return &E.mus[2 * SIM_MUS_CA * SIM_MUS_STRIDE + b * 6]; }

// sum copies 1..nc-1 of table t (tables of nc copies each) into its copy 0
template <class L>
__device__ __forceinline__ void mus_fold(L& E, int t, int nc, int ln) {
  real* base = &E.mus[t * nc * SIM_MUS_STRIDE];
  for (int e = ln; e < SIM_MAXJ * 6; e += SIM_WAVE) {
    real s = base[e];
    for (int c = 1; c < nc; ++c) s += base[c * SIM_MUS_STRIDE + e];
    base[e] = s;
  }
}

template <class L>
__device__ __forceinline__ void muscle_wrenches(const Scal* __restrict__ m, L& E, int ln) {
  for (int i = ln; i < SIM_MUS_CF * SIM_MUS_STRIDE; i += SIM_WAVE) E.mus[i] = RL(0.0);
  wsync();
  real* fm = &E.mus[(ln % SIM_MUS_CF) * SIM_MUS_STRIDE];
  SIM_PHASE(E, PH_F_MUSCLE);
  for (int i0 = 0; i0 < m->n_mtu; i0 += SIM_WAVE) {
    const int i = i0 + ln;
    if (i < m->n_mtu) {
      MtuPath P;
      mtu_path(m, E, i, P, E.act[i]);
      SIM_PHASE(E, PH_FM_PATH);
      // consecutive points on one body are summed first: one addition per run of points
      sv acc = zsv();
      int cur = P.b[0];
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT; ++k) {
        if (k < P.np) {
          const sv w = spf(P.x[k], scl3(mtu_udiff(P, k), P.F));
          if (P.b[k] != cur) {
            lds_add6(fm + cur * 6, acc);
            acc = w;
            cur = P.b[k];
          } else {
            acc = addsv(acc, w);
          }
        }
      }
      lds_add6(fm + cur * 6, acc);
      SIM_PHASE(E, PH_FM_ACC);
    }
  }
  wsync();
  mus_fold(E, 0, SIM_MUS_CF, ln);
  wsync();
}

// Adjoint of the muscle forces in lambda^T ID = ... - sum_p nu_p . f_p (nu_p the virtual
// velocity of point p under lambda): recomputes the tensions and the wrench table, adds to E.act_bar
// the activation term, and collects per body the terms of the point-force adjoint that the
// contacts use (mus_ab: Sp(x, xbar) + (-nu x f + v x vbar, 0); mus_vb: Sp(x, vbar)), where
// xbar, vbar are the derivatives of F delta (delta = sum u_k . (nu_{k+1} - nu_k)) through
// the tension and the segment directions.
template <class L>
__device__ __forceinline__ void muscle_adjoint(const Scal* __restrict__ m, L& E, int ln) {
  for (int i = ln; i < 3 * SIM_MUS_CA * SIM_MUS_STRIDE; i += SIM_WAVE) E.mus[i] = RL(0.0);
  wsync();
  // lane l adds into copy l % SIM_MUS_CA of each table (see muscle_wrenches)
  const int cp = ln % SIM_MUS_CA;
  real* fm = &E.mus[cp * SIM_MUS_STRIDE];
  real* mab = &E.mus[(SIM_MUS_CA + cp) * SIM_MUS_STRIDE];
  real* mvb = &E.mus[(2 * SIM_MUS_CA + cp) * SIM_MUS_STRIDE];
  SIM_PHASE(E, PH_A_MUSCLE);
  for (int i0 = 0; i0 < m->n_mtu; i0 += SIM_WAVE) {
    const int i = i0 + ln;
    if (i < m->n_mtu) {
      const real act = E.act[i];
      MtuPath P;
      mtu_path(m, E, i, P, act);
      SIM_PHASE(E, PH_AM_PATH);
      f3 nu[SIM_MAXMPT];
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT; ++k) nu[k] = ptv(ldsv(E.W[P.b[k]]), P.x[k]);
      real delta = RL(0.0);
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT - 1; ++k)
        if (k + 1 < P.np) delta += dot3(P.u[k], sub3(nu[k + 1], nu[k]));
      // at zero raw tension (e.g. zero activation) the derivative is the active branch's
      const bool on = P.Fr >= RL(0.0);
      const real lopt = P.lopt, fmax = P.fmax;
      const real z = (P.lt - RL(1.0)) / m->fl_w;
      const real dFdL = on ? fmax * act * P.fv * P.fl * (-RL(2.0) * z / m->fl_w) / lopt : RL(0.0);
      const real dFdLd = on ? fmax * act * P.fl / (m->vmax * lopt) : RL(0.0);
      const real dFda = on ? fmax * P.fl * P.fv : RL(0.0);
      E.act_bar[i] -= delta * dFda;
      const real cL = dFdL * delta, cV = dFdLd * delta;
      f3 xb[SIM_MAXMPT];
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT; ++k) xb[k] = scl3(mtu_udiff(P, k), -cL);
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT - 1; ++k) {
        if (k + 1 < P.np) {
          // d(u_k . a)/dx_{k+1} = (a - u_k (u_k . a)) / l_k
          f3 dv = sub3(P.v[k + 1], P.v[k]), dn = sub3(nu[k + 1], nu[k]);
          f3 pv = sub3(dv, scl3(P.u[k], dot3(P.u[k], dv)));
          f3 pn = sub3(dn, scl3(P.u[k], dot3(P.u[k], dn)));
          f3 g = scl3(add3(scl3(pv, cV), scl3(pn, P.F)), P.il[k]);
          xb[k + 1] = add3(xb[k + 1], g);
          xb[k] = sub3(xb[k], g);
        }
      }
      SIM_PHASE(E, PH_AM_DERIV);
      // consecutive points on one body are summed first (see muscle_wrenches)
      sv af = zsv(), aa = zsv(), av = zsv();
      int cur = P.b[0];
#pragma unroll
      for (int k = 0; k < SIM_MAXMPT; ++k) {
        if (k < P.np) {
          const f3 ud = mtu_udiff(P, k);
          const f3 f = scl3(ud, P.F);
          const f3 vb = scl3(ud, -cV);
          const sv wf = spf(P.x[k], f);
          const sv wa = addsv(spf(P.x[k], xb[k]),
                              mksv(add3(scl3(cross3(nu[k], f), -RL(1.0)), cross3(P.v[k], vb)),
                                   mk3(RL(0.0), RL(0.0), RL(0.0))));
          const sv wv = spf(P.x[k], vb);
          if (P.b[k] != cur) {
            lds_add6(fm + cur * 6, af);
            lds_add6(mab + cur * 6, aa);
            lds_add6(mvb + cur * 6, av);
            af = wf; aa = wa; av = wv;
            cur = P.b[k];
          } else {
            af = addsv(af, wf); aa = addsv(aa, wa); av = addsv(av, wv);
          }
        }
      }
      lds_add6(fm + cur * 6, af);
      lds_add6(mab + cur * 6, aa);
      lds_add6(mvb + cur * 6, av);
      SIM_PHASE(E, PH_AM_ACC);
    }
  }
  wsync();
  for (int t = 0; t < 3; ++t) mus_fold(E, t, SIM_MUS_CA, ln);
  wsync();
}

// Kinematics and contacts of the substep (the part of the forward that the reverse reads back,
// besides the factor and the accelerations): reference point, joint rotations, frame
// transforms, screws, velocities and bias accelerations, contact forces.  Leaves the lane's
// frame rotation and position in R, p and its screw, velocity and bias acceleration in S, v, ab.
template <class L>
__device__ __forceinline__ void substep_kin(const Scal* __restrict__ m, L& E, const JointRegs& jr,
                                            const ContactRegs& cr, int ln, real* R, f3& p, sv& S, sv& v, sv& ab) {
  constexpr int LN = L::kLanes;
  const int J = m->J, nc = m->nc;
  const real g = m->g;
  // reference point O = root position (floating) or world origin
  if (ln < 3) E.O[ln] = m->floating ? E.q[ln] : RL(0.0);
  wsync();
  // ---- local joint rotations (all lanes at once), then kinematics, velocities and bias
  // accelerations along the root paths; each lane keeps its own frame's results in registers
  real Rot[9];
  real qj = RL(0.0), qdj = RL(0.0);
  if (ln < J) {
    if (jr.type == J_FREE) {
      quat_rot(E.q[jr.qa + 3], E.q[jr.qa + 4], E.q[jr.qa + 5], E.q[jr.qa + 6], Rot);
    } else {
      qj = E.q[jr.qa];
      qdj = E.qd[jr.va];
      if (jr.type == J_HINGE) {
        real sn, cs;
        m_sincos(qj, &sn, &cs);
        real omc = RL(1.0) - cs;
        f3 a = ld3(E.j_ax[ln]);
        // Rodrigues: Rot = I + sn K + (1 - cs) K^2 with K = [a]x, K^2 = a a^T - I
        Rot[0] = RL(1.0) + omc * (a.x * a.x - RL(1.0)); Rot[1] = -sn * a.z + omc * a.x * a.y; Rot[2] = sn * a.y + omc * a.x * a.z;
        Rot[3] = sn * a.z + omc * a.y * a.x; Rot[4] = RL(1.0) + omc * (a.y * a.y - RL(1.0)); Rot[5] = -sn * a.x + omc * a.y * a.z;
        Rot[6] = -sn * a.y + omc * a.z * a.x; Rot[7] = sn * a.x + omc * a.z * a.y; Rot[8] = RL(1.0) + omc * (a.z * a.z - RL(1.0));
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Rot[k] = (k % 4 == 0) ? RL(1.0) : RL(0.0);
      }
    }
  }
  S = zsv();
  int rounds = 0;
  while ((1 << rounds) <= m->max_depth) ++rounds;
  {
    // Frame transforms by pointer jumping.  Each frame starts from its transform relative
    // to its parent (rotation Rot, translation t) and a link to the parent; a round
    // composes the frame's partial path with the partial path of the frame its link names
    // and takes over that frame's link, so after ceil(log2(max_depth + 1)) rounds every
    // frame holds its whole root path.  A round's values come from the other lanes'
    // registers before the round (wavefront permutes).
    f3 t = mk3(RL(0.0), RL(0.0), RL(0.0));
    if (ln < J && jr.type != J_FREE) {
      t = ld3(E.j_off[ln]);
      if (jr.type == J_SLIDE) t = add3(t, scl3(ld3(E.j_ax[ln]), qj));
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (ln < J) ? Rot[k] : ((k % 4 == 0) ? RL(1.0) : RL(0.0));
    p = t;
    int link = (ln < J) ? jr.par : -1;
    for (int r = 0; r < rounds; ++r) {
      const int src = link >= 0 ? link : ln;
      real Ra[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Ra[k] = pull_g<LN>(R[k], src);
      const f3 pa = mk3(pull_g<LN>(p.x, src), pull_g<LN>(p.y, src), pull_g<LN>(p.z, src));
      const int nl = pull_g<LN>(link, src);
      if (link >= 0) {
        real Rn[9];
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            Rn[3 * rr + c] = Ra[3 * rr] * R[c] + Ra[3 * rr + 1] * R[3 + c] + Ra[3 * rr + 2] * R[6 + c];
        p = add3(pa, mv3(Ra, p));
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = Rn[k];
        link = nl;
      }
    }
  }
  SIM_PHASE(E, PH_F_FK);
  // motion subspaces: a hinge turns about its own axis, so its world axis is R ax either
  // side of the joint rotation; a slide keeps the parent's rotation
  sv u = zsv(), c = zsv();
  if (ln < J) {
    if (jr.type == J_FREE) {
      f3 vl = mk3(E.qd[jr.va], E.qd[jr.va + 1], E.qd[jr.va + 2]);
      f3 w = mk3(E.qd[jr.va + 3], E.qd[jr.va + 4], E.qd[jr.va + 5]);
      u = mksv(w, vl);
      c = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), add3(mk3(RL(0.0), RL(0.0), g), cross3(vl, w)));
    } else {
      f3 sh = mv3(R, ld3(E.j_ax[ln]));
      S = (jr.type == J_HINGE) ? mksv(sh, cross3(p, sh)) : mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), sh);
      u = sclsv(S, qdj);
    }
  }
  // velocities v_j = sum of u_k = S_k qd_k over the root path and bias accelerations
  // ab_j = sum of v_k x u_k over the path (plus gravity at the root), in one pointer-jumping
  // pass: for a path segment (V, C) = (sum u, sum of v x u with v measured from the
  // segment's top), appending the segment below gives V = Va + Vb, C = Ca + Cb + Va x Vb
  // (u x u = 0, so a single frame starts from C = 0)
  {
    sv V = u, Cs = zsv();
    if (ln < J) {
      if (jr.type == J_FREE) Cs = c;
      else if (jr.par < 0) Cs = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), mk3(RL(0.0), RL(0.0), g));
    }
    int link = (ln < J) ? jr.par : -1;
    for (int r = 0; r < rounds; ++r) {
      const int src = link >= 0 ? link : ln;
      const sv Va = pull_sv<LN>(V, src);
      const sv Ca = pull_sv<LN>(Cs, src);
      const int nl = pull_g<LN>(link, src);
      if (link >= 0) {
        Cs = addsv(addsv(Ca, Cs), crm(Va, V));
        V = addsv(Va, V);
        link = nl;
      }
    }
    v = V;
    ab = Cs;
  }
  if (ln < J) {
#pragma unroll
    for (int k = 0; k < 9; ++k) E.R[ln][k] = R[k];
    st3(E.p[ln], p);
    stsv(E.S[ln], S);
    stsv(E.v[ln], v);
    stsv(E.ab[ln], ab);
  }
  wsync();
  SIM_PHASE(E, PH_F_VEL);
  // ---- contacts (lane = contact)
  bool adh = false;
  if (ln < nc) {
    int b = cr.body;
    f3 xc = add3(ld3(E.p[b]), mv3(E.R[b], cr.pos));
    f3 xp = mk3(xc.x, xc.y, xc.z - cr.rad);
    real d = xc.z + E.O[2] - cr.rad;
    f3 vpt = ptv(ldsv(E.v[b]), xp);
    f3 dd;
    real dv[9];
    f3 f = contact_force(m, d, vpt, false, &dd, dv);
    st3(E.cf[ln], f);
    st3(E.cx[ln], xp);
    st3(E.cvel[ln], vpt);
    E.cdep[ln] = d;
    // the literal damping term makes a penetrating contact pull when d_dot > k_n / k_d
    adh = (d < RL(0.0)) && (f.z < RL(0.0));
  }
  {
    const unsigned long long bal = grp_ballot<LN>(adh);
    if (ln == 0) E.nadh = __popcll(bal);
  }
  wsync();
  SIM_PHASE(E, PH_F_CONTACT);
}

// The world spatial inertia (10 numbers) of the lane's body from its frame R, p.
template <class L>
__device__ __forceinline__ void body_inertia(const L& E, const JointRegs& jr, int ln, const real* R, f3 p,
                                             real* Ib) {
  real mass = jr.mass;
  f3 c = add3(p, mv3(R, ld3(E.j_com[ln])));
  // Ic_w = R I R^T
  const real* I6 = E.j_I6[ln];
  real Il[9] = {I6[0], I6[3], I6[4], I6[3], I6[1], I6[5], I6[4], I6[5], I6[2]};
  real T[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) T[3 * r + k] = R[3 * r] * Il[k] + R[3 * r + 1] * Il[3 + k] + R[3 * r + 2] * Il[6 + k];
  real Iw[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) Iw[3 * r + k] = T[3 * r] * R[3 * k] + T[3 * r + 1] * R[3 * k + 1] + T[3 * r + 2] * R[3 * k + 2];
  real cc = dot3(c, c);
  Ib[0] = mass;
  Ib[1] = mass * c.x; Ib[2] = mass * c.y; Ib[3] = mass * c.z;
  Ib[4] = Iw[0] + mass * (cc - c.x * c.x);
  Ib[5] = Iw[4] + mass * (cc - c.y * c.y);
  Ib[6] = Iw[8] + mass * (cc - c.z * c.z);
  Ib[7] = Iw[1] - mass * c.x * c.y;
  Ib[8] = Iw[2] - mass * c.x * c.z;
  Ib[9] = Iw[5] - mass * c.y * c.z;
}

// Positions from the new velocities E.qdn (semi-implicit Euler; the free root's orientation
// by the exact exponential map) into E.qn, and the muscle activations into E.actn.
template <class L>
__device__ __forceinline__ void integrate_positions(const Scal* __restrict__ m, L& E, const JointRegs& jr, int ln) {
  const real dt = m->dt_sub;
  const int J = m->J;
  // ---- positions with the new velocities (lane = joint)
  if (ln < J) {
    if (jr.type == J_FREE) {
      int qa = jr.qa, va = jr.va;
#pragma unroll
      for (int k = 0; k < 3; ++k) E.qn[qa + k] = E.q[qa + k] + dt * E.qdn[va + k];
      f3 w = mk3(E.qdn[va + 3], E.qdn[va + 4], E.qdn[va + 5]);
      real c, s, dc, ds;
      dq_coeffs(dot3(w, w), RL(0.5) * dt, c, s, dc, ds);
      real a0 = c, a1 = s * w.x, a2 = s * w.y, a3 = s * w.z;
      real b0 = E.q[qa + 3], b1 = E.q[qa + 4], b2 = E.q[qa + 5], b3 = E.q[qa + 6];
      E.qn[qa + 3] = a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3;
      E.qn[qa + 4] = a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2;
      E.qn[qa + 5] = a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1;
      E.qn[qa + 6] = a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0;
    } else {
      E.qn[jr.qa] = E.q[jr.qa] + dt * E.qdn[jr.va];
    }
  }
  if constexpr (L::kMtu > 0) {
    // activation lag, explicit with the pre-substep activation
    const real ka = dt / m->tau_act;
    for (int i = ln; i < m->n_mtu; i += SIM_WAVE) E.actn[i] = E.act[i] + ka * (E.a[m->n_motor + i] - E.act[i]);
  }
}

template <int NV, class L>
__device__ __forceinline__ void substep_forward(const Scal* __restrict__ m, L& E,
                                                const JointRegs& jr, const ContactRegs& cr, int ln,
                                                Chol& C, bool inplace, int& fb) {
  constexpr int LN = L::kLanes;
  const int J = m->J, nv = m->nv;
  const real dt = m->dt_sub;
  // clear M
  for (int i = ln; i < L::kV * (L::kV + 1); i += LN) (&E.M[0][0])[i] = RL(0.0);
  real R[9];
  f3 p;
  sv S, v, ab;
  substep_kin(m, E, jr, cr, ln, R, p, S, v, ab);
  if constexpr (L::kMtu > 0) {
    muscle_wrenches(m, E, ln);
    SIM_PHASE(E, PH_F_MUSCLE);
  }
  // ---- body inertias and Newton-Euler forces (lane = joint), joint torques
  if (ln < J) {
    real Ib[10];
    body_inertia(E, jr, ln, R, p, Ib);
#pragma unroll
    for (int k = 0; k < 10; ++k) { E.Ib[ln][k] = Ib[k]; E.Ic[ln][k] = Ib[k]; }
    sv hv = iapply(Ib, v);
    sv f = addsv(iapply(Ib, ab), crf(v, hv));
    for (unsigned int cm = jr.cmask; cm; cm &= cm - 1) {
      int ci = __builtin_ctz(cm);
      f = subsv(f, spf(ld3(E.cx[ci]), ld3(E.cf[ci])));
    }
    if constexpr (L::kMtu > 0) f = subsv(f, ldsv(mus_fm(E, ln)));
    stsv(E.F[ln], f);
    // joint torques: actuation + limit penalty
    if (jr.type != J_FREE) {
      real tau = RL(0.0);
      if (jr.act >= 0) tau = jr.gear * E.a[jr.act];
      if (jr.lim) {
        real qj = E.q[jr.qa];
        if (qj < jr.lo) tau += m->klim * (jr.lo - qj);
        else if (qj > jr.hi) tau += m->klim * (jr.hi - qj);
      }
      E.vec[jr.va] = tau;
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) E.vec[jr.va + k] = RL(0.0);
    }
  }
  wsync();
  SIM_PHASE(E, PH_F_NE);
  // ---- subtree sums of forces (6 columns) and composite inertias (10 columns)
  tree_sum_sched16(E, m->ts_steps, ln);
  wsync();
  SIM_PHASE(E, PH_F_TREESUM);
  // ---- bias into rhs; composite-inertia columns F_i = Ic_i S_i; root block of M
  if (ln < J) {
    sv F = ldsv(E.F[ln]);
    const real* Ic = E.Ic[ln];
    if (jr.type == J_FREE) {
      int va = jr.va;
      E.vec[va + 0] -= F.l.x; E.vec[va + 1] -= F.l.y; E.vec[va + 2] -= F.l.z;
      E.vec[va + 3] -= F.a.x; E.vec[va + 4] -= F.a.y; E.vec[va + 5] -= F.a.z;
      real m0 = Ic[0];
      f3 h = mk3(Ic[1], Ic[2], Ic[3]);
      real Ibar[9] = {Ic[4], Ic[7], Ic[8], Ic[7], Ic[5], Ic[9], Ic[8], Ic[9], Ic[6]};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
#pragma unroll
        for (int f2 = 0; f2 < 3; ++f2) {
          E.M[va + e][va + f2] = (e == f2) ? m0 : RL(0.0);
          E.M[va + 3 + e][va + 3 + f2] = Ibar[3 * e + f2];
        }
      }
      // M[v_e][w_f] = (e_f x h)_e
      f3 ex = cross3(mk3(1, 0, 0), h), ey = cross3(mk3(0, 1, 0), h), ez = cross3(mk3(0, 0, 1), h);
      real C[9] = {ex.x, ey.x, ez.x, ex.y, ey.y, ez.y, ex.z, ey.z, ez.z};
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int f2 = 0; f2 < 3; ++f2) {
          E.M[va + e][va + 3 + f2] = C[3 * e + f2];
          E.M[va + 3 + f2][va + e] = C[3 * e + f2];
        }
    } else {
      E.vec[jr.va] -= dotsv(S, F);
      stsv(E.Fi[ln], iapply(Ic, S));
    }
  }
  wsync();
  SIM_PHASE(E, PH_F_BIAS);
  // ---- CRBA entries M[va_k][va_i] = S_k . F_i, one (frame, ancestor) pair per lane and round
  for (int r = 0; r * LN < jr.npair; ++r) {
    int pi = r * LN + ln;
    int pk = pi < jr.npair ? E.pairs[pi] : 0;
    if (pk) {
      int i = pk & 31, k = (pk >> 5) & 31, vi = (pk >> 10) & 31, vk = (pk >> 15) & 31;
      sv Fi = ldsv(E.Fi[i]);
      if (pk & (1 << 20)) {
        E.M[vk + 0][vi] = Fi.l.x; E.M[vk + 1][vi] = Fi.l.y; E.M[vk + 2][vi] = Fi.l.z;
        E.M[vk + 3][vi] = Fi.a.x; E.M[vk + 4][vi] = Fi.a.y; E.M[vk + 5][vi] = Fi.a.z;
        E.M[vi][vk + 0] = Fi.l.x; E.M[vi][vk + 1] = Fi.l.y; E.M[vi][vk + 2] = Fi.l.z;
        E.M[vi][vk + 3] = Fi.a.x; E.M[vi][vk + 4] = Fi.a.y; E.M[vi][vk + 5] = Fi.a.z;
      } else {
        real mk = dotsv(ldsv(E.S[k]), Fi);
        if (k == i) mk += E.arm[vi];
        E.M[vk][vi] = mk;
        E.M[vi][vk] = mk;
      }
    }
  }
  wsync();
  SIM_PHASE(E, PH_F_CRBA);
  // ---- Cholesky and solve (lane = DOF); rows >= nv padded with the identity
  if (nv == NV) {
    // no padding: the lanes past the matrix read row 0; no lane of the matrix reads them back
#pragma unroll
    for (int k = 0; k < NV; ++k) C.row[k] = E.M[ln < nv ? ln : 0][k];
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      C.row[k] = (ln < nv && k < nv) ? E.M[ln < nv ? ln : 0][k] : ((ln == k) ? RL(1.0) : RL(0.0));
  }
  real minpiv;
  real dmax = grp_max<LN>(ln < nv ? E.M[ln < nv ? ln : 0][ln < nv ? ln : 0] : RL(0.0));
  chol_factor<NV, LN>(C, ln, minpiv);
  fb = 0;
  if (sizeof(real) == 4 && !(minpiv > m->chol_thr * dmax)) fb = 1;
  real b = ln < nv ? E.vec[ln] : RL(0.0);
  real x;
  SIM_PHASE(E, PH_F_CHOL);
  if (fb) {
    chol64_factor<NV>(E, nv, ln);
    SIM_PHASE(E, PH_F_FACTOR);
    x = (real)chol64_solve<NV>(E, ln, (double)b);
  } else {
    wsync();
    if (ln < NV) {
#pragma unroll
      for (int k = 0; k < NV; ++k) E.M[ln][k] = C.row[k];   // padded rows hold the identity
    }
    wsync();
    const int lc = ln < NV ? ln : 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) C.col[k] = (ln < NV) ? E.M[k][lc] : RL(0.0);
    SIM_PHASE(E, PH_F_FACTOR);
    x = chol_solve<NV, LN>(C, ln, b);
  }
  if (ln < nv) {
    E.qdd[ln] = x;
    real qdn = E.qd[ln] + dt * x;
    E.qdn[ln] = qdn;
  }
  wsync();
  SIM_PHASE(E, PH_F_SOLVE);
  integrate_positions(m, E, jr, ln);
  wsync();
  if (inplace) {
    if (ln < m->nq) E.q[ln] = E.qn[ln];
    if (ln < nv) E.qd[ln] = E.qdn[ln];
    if constexpr (L::kMtu > 0)
      for (int i = ln; i < m->n_mtu; i += SIM_WAVE) E.act[i] = E.actn[i];
    wsync();
  }
  SIM_PHASE(E, PH_F_INTEG);
}

// What the reverse of a substep reads of its forward when the factor and the accelerations
// come from the factor cache: the kinematics, the contacts and the body inertias of the
// pre-substep state, computed by the forward's own code.
template <class L>
__device__ __forceinline__ void substep_kinematics(const Scal* __restrict__ m, L& E, const JointRegs& jr,
                                                   const ContactRegs& cr, int ln) {
  real R[9];
  f3 p;
  sv S, v, ab;
  substep_kin(m, E, jr, cr, ln, R, p, S, v, ab);
  if (ln < m->J) {
    real Ib[10];
    body_inertia(E, jr, ln, R, p, Ib);
#pragma unroll
    for (int k = 0; k < 10; ++k) E.Ib[ln][k] = Ib[k];
  }
  wsync();
  SIM_PHASE(E, PH_F_NE);
}

// --------------------------------------------------------------- adjoint of one substep
// On entry E.q/E.qd/E.a hold the pre-substep state, E.qb/E.qdb the adjoint of the
// post-substep state.  On exit E.qb/E.qdb hold the adjoint of the pre-substep state and
// E.abar has gained this substep's contribution.
template <int NV, class L>
__device__ __forceinline__ void substep_adjoint_core(const Scal* __restrict__ m, L& E,
                                                     const JointRegs& jr, const ContactRegs& cr, int ln,
                                                     const Chol& C, int fb) {
  constexpr int LN = L::kLanes;
  const int J = m->J, nv = m->nv, nc = m->nc;
  const real dt = m->dt_sub;
  const real g = m->g;
  if constexpr (L::kMtu > 0) {
    // activation lag reverse: act' = act + (dt/tau)(u - act)
    const real ka = dt / m->tau_act;
    for (int i = ln; i < m->n_mtu; i += SIM_WAVE) {
      const real gb = E.act_bar[i];
      E.abar[m->n_motor + i] += ka * gb;
      E.act_bar[i] = gb - ka * gb;
    }
  }
  // ---- integrator reverse (lane = joint)
  if (ln < J) {
    if (jr.type == J_FREE) {
      int qa = jr.qa, va = jr.va;
#pragma unroll
      for (int k = 0; k < 3; ++k) E.qdb[va + k] += dt * E.qb[qa + k];
      f3 w = mk3(E.qdn[va + 3], E.qdn[va + 4], E.qdn[va + 5]);
      real c, s, dc, ds;
      dq_coeffs(dot3(w, w), RL(0.5) * dt, c, s, dc, ds);
      real d0 = c, d1 = s * w.x, d2 = s * w.y, d3 = s * w.z;
      real b0 = E.q[qa + 3], b1 = E.q[qa + 4], b2 = E.q[qa + 5], b3 = E.q[qa + 6];
      real g0 = E.qb[qa + 3], g1 = E.qb[qa + 4], g2 = E.qb[qa + 5], g3 = E.qb[qa + 6];
      // quat' = L(dq) quat  ->  quat_bar = L(dq)^T quat'_bar
      real q0 = d0 * g0 + d1 * g1 + d2 * g2 + d3 * g3;
      real q1 = -d1 * g0 + d0 * g1 + d3 * g2 - d2 * g3;
      real q2 = -d2 * g0 - d3 * g1 + d0 * g2 + d1 * g3;
      real q3 = -d3 * g0 + d2 * g1 - d1 * g2 + d0 * g3;
      // quat' = Rm(quat) dq  ->  dq_bar = Rm(quat)^T quat'_bar
      real e0 = b0 * g0 + b1 * g1 + b2 * g2 + b3 * g3;
      real e1 = -b1 * g0 + b0 * g1 - b3 * g2 + b2 * g3;
      real e2 = -b2 * g0 + b3 * g1 + b0 * g2 - b1 * g3;
      real e3 = -b3 * g0 - b2 * g1 + b1 * g2 + b0 * g3;
      f3 ev = mk3(e1, e2, e3);
      f3 wbar = add3(add3(scl3(w, RL(2.0) * dc * e0), scl3(ev, s)), scl3(w, RL(2.0) * ds * dot3(w, ev)));
      E.qdb[va + 3] += wbar.x; E.qdb[va + 4] += wbar.y; E.qdb[va + 5] += wbar.z;
      E.qb[qa + 3] = q0; E.qb[qa + 4] = q1; E.qb[qa + 5] = q2; E.qb[qa + 6] = q3;
    } else {
      E.qdb[jr.va] += dt * E.qb[jr.qa];
    }
  }
  wsync();
  SIM_PHASE(E, PH_A_INTEG);
  // ---- lambda = M^{-1} qdd_bar with the cached factor (lane = DOF)
  {
    real rb = ln < nv ? dt * E.qdb[ln] : RL(0.0);
    real lam = fb ? (real)chol64_solve<NV>(E, ln, (double)rb) : chol_solve<NV, LN>(C, ln, rb);
    if (ln < nv) E.lam[ln] = lam;
  }
  wsync();
  SIM_PHASE(E, PH_A_LAMBDA);
  // actuation adjoint and full accelerations / virtual velocities
  if (ln < J && jr.act >= 0) E.abar[jr.act] += jr.gear * E.lam[jr.va];
  // local terms (lane = joint), then their sums along each root path by pointer jumping
  sv A = zsv(), W = zsv();
  if (ln < J) {
    if (jr.type == J_FREE) {
      int va = jr.va;
      sv ab = ldsv(E.ab[ln]);
      A = addsv(ab, mksv(mk3(E.qdd[va + 3], E.qdd[va + 4], E.qdd[va + 5]),
                         mk3(E.qdd[va], E.qdd[va + 1], E.qdd[va + 2])));
      W = mksv(mk3(E.lam[va + 3], E.lam[va + 4], E.lam[va + 5]), mk3(E.lam[va], E.lam[va + 1], E.lam[va + 2]));
    } else {
      sv S = ldsv(E.S[ln]);
      sv v = ldsv(E.v[ln]);
      sv u = sclsv(S, E.qd[jr.va]);
      A = addsv(sclsv(S, E.qdd[jr.va]), crm(v, u));
      W = sclsv(S, E.lam[jr.va]);
      if (jr.par < 0) A = addsv(A, mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), mk3(RL(0.0), RL(0.0), g)));
    }
  }
  {
    int rounds = 0;
    while ((1 << rounds) <= m->max_depth) ++rounds;
    path_sum2<LN>(A, W, (ln < J) ? jr.par : -1, rounds);
  }
  if (ln < J) {
    stsv(E.A[ln], A);
    stsv(E.W[ln], W);
  }
  wsync();
  SIM_PHASE(E, PH_A_PATH);
  // ---- contact adjoints (lane = contact)
  if (ln < nc) {
    int b = cr.body;
    f3 x = ld3(E.cx[ln]);
    f3 vpt = ld3(E.cvel[ln]);
    f3 f = ld3(E.cf[ln]);
    sv Wb = ldsv(E.W[b]);
    sv vb = ldsv(E.v[b]);
    f3 nu = ptv(Wb, x);
    f3 dfdd;
    real dfdv[9];
    contact_force(m, E.cdep[ln], vpt, true, &dfdd, dfdv);
    f3 fbar = scl3(nu, -RL(1.0));
    f3 xbar = mk3(RL(0.0), RL(0.0), dot3(dfdd, fbar));
    f3 vbar = mk3(dfdv[0] * fbar.x + dfdv[3] * fbar.y + dfdv[6] * fbar.z,
                  dfdv[1] * fbar.x + dfdv[4] * fbar.y + dfdv[7] * fbar.z,
                  dfdv[2] * fbar.x + dfdv[5] * fbar.y + dfdv[8] * fbar.z);
    f3 r = mk3(RL(0.0), RL(0.0), cr.rad);
    f3 extra = cross3(r, sub3(add3(xbar, cross3(vbar, vb.a)), cross3(f, Wb.a)));
    sv ab = addsv(spf(x, xbar), mksv(add3(add3(scl3(cross3(nu, f), -RL(1.0)), cross3(vpt, vbar)), extra),
                                    mk3(RL(0.0), RL(0.0), RL(0.0))));
    stsv(E.cAb[ln], ab);
    stsv(E.cVb[ln], spf(x, vbar));
  }
  wsync();
  SIM_PHASE(E, PH_A_CONTACT);
  if constexpr (L::kMtu > 0) {
    muscle_adjoint(m, E, ln);
    SIM_PHASE(E, PH_A_MUSCLE);
  }
  // ---- per-body terms (lane = joint): P Q R T Fn Ab Vb
  if (ln < J) {
    const real* Ib = E.Ib[ln];
    sv v = ldsv(E.v[ln]), W = ldsv(E.W[ln]), A = ldsv(E.A[ln]);
    sv Iw = iapply(Ib, W);
    sv hv = iapply(Ib, v);
    sv Q = crf(v, Iw);
    sv Rr = crf(W, hv);
    sv T = iapply(Ib, crm(v, W));
    sv Fn = addsv(iapply(Ib, A), crf(v, hv));
    sv Ab = zsv(), Vb = zsv();
    for (unsigned int cm = jr.cmask; cm; cm &= cm - 1) {
      int ci = __builtin_ctz(cm);
      Fn = subsv(Fn, spf(ld3(E.cx[ci]), ld3(E.cf[ci])));
      Ab = addsv(Ab, ldsv(E.cAb[ci]));
      Vb = addsv(Vb, ldsv(E.cVb[ci]));
    }
    if constexpr (L::kMtu > 0) {
      Fn = subsv(Fn, ldsv(mus_fm(E, ln)));
      Ab = addsv(Ab, ldsv(mus_ab(E, ln)));
      Vb = addsv(Vb, ldsv(mus_vb(E, ln)));
    }
    real* o = E.acc[ln];
    stsv(o + 0, Iw); stsv(o + 6, Q); stsv(o + 12, Rr); stsv(o + 18, T);
    stsv(o + 24, Fn); stsv(o + 30, Ab); stsv(o + 36, Vb);
  }
  wsync();
  SIM_PHASE(E, PH_A_BODY);
  // one lane per column of the 42 (several passes with fewer than 42 lanes per environment)
#pragma unroll
  for (int c0 = 0; c0 < 42; c0 += LN) {
    const int c = c0 + ln;
    tree_sum_cols(&E.acc[0][c < 42 ? c : 0], 42, c < 42, J, jr.par);
  }
  wsync();
  SIM_PHASE(E, PH_A_TREESUM);
  // ---- derivatives of lambda^T ID per joint (lane = joint)
  if (ln < J) {
    const real* o = E.acc[ln];
    sv P = ldsv(o + 0), Q = ldsv(o + 6), Rr = ldsv(o + 12), T = ldsv(o + 18);
    sv Fn = ldsv(o + 24), Ab = ldsv(o + 30), Vb = ldsv(o + 36);
    sv QRT = subsv(subsv(Q, Rr), T);
    if (jr.type == J_FREE) {
      int va = jr.va;
      sv vA = ldsv(E.v[ln]), wA = ldsv(E.W[ln]), aA = ldsv(E.A[ln]);
      f3 vl = mk3(E.qd[va], E.qd[va + 1], E.qd[va + 2]);
      f3 w = mk3(E.qd[va + 3], E.qd[va + 4], E.qd[va + 5]);
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        f3 ue = mk3(e == 0 ? RL(1.0) : RL(0.0), e == 1 ? RL(1.0) : RL(0.0), e == 2 ? RL(1.0) : RL(0.0));
        sv Te = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), ue);
        sv Se = mksv(ue, mk3(RL(0.0), RL(0.0), RL(0.0)));
        E.dPq[va + e] = dotsv(Te, Ab);
        sv ee = crm(Se, vA);
        E.dPq[va + 3 + e] = -dotsv(crm(Se, wA), Fn) - dotsv(crm(Se, aA), P) - dotsv(ee, Q) +
                            dotsv(crm(ee, vA), P) + dotsv(ee, Rr) + dotsv(ee, T) + dotsv(Se, Ab) - dotsv(ee, Vb);
        sv daT = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), cross3(ue, w));
        sv daS = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), cross3(vl, ue));
        E.dPqd[va + e] = dotsv(Te, QRT) - dotsv(crm(Te, vA), P) + dotsv(daT, P) + dotsv(Te, Vb);
        E.dPqd[va + 3 + e] = dotsv(Se, QRT) - dotsv(crm(Se, vA), P) + dotsv(daS, P) + dotsv(Se, Vb);
      }
    } else {
      sv S = ldsv(E.S[ln]);
      sv vA, wA, aA;
      if (jr.par >= 0) {
        vA = ldsv(E.v[jr.par]); wA = ldsv(E.W[jr.par]); aA = ldsv(E.A[jr.par]);
      } else {
        vA = zsv(); wA = zsv(); aA = mksv(mk3(RL(0.0), RL(0.0), RL(0.0)), mk3(RL(0.0), RL(0.0), g));
      }
      sv ee = crm(S, vA);
      real val = -dotsv(crm(S, wA), Fn) - dotsv(crm(S, aA), P) - dotsv(ee, Q) + dotsv(crm(ee, vA), P) +
                  dotsv(ee, Rr) + dotsv(ee, T) + dotsv(S, Ab) - dotsv(ee, Vb);
      if (jr.lim) {
        real qj = E.q[jr.qa];
        if (qj < jr.lo || qj > jr.hi) val += E.lam[jr.va] * m->klim;
      }
      E.dPq[jr.va] = val;
      E.dPqd[jr.va] = dotsv(S, QRT) - RL(2.0) * dotsv(ee, P) + dotsv(S, Vb);
    }
  }
  wsync();
  SIM_PHASE(E, PH_A_DERIV);
  // ---- adjoint of the pre-substep state
  if (ln < nv) E.qdb[ln] -= E.dPqd[ln];
  if (ln < J) {
    if (jr.type == J_FREE) {
      int qa = jr.qa, va = jr.va;
#pragma unroll
      for (int k = 0; k < 3; ++k) E.qb[qa + k] -= E.dPq[va + k];
      f3 tr = mk3(E.dPq[va + 3], E.dPq[va + 4], E.dPq[va + 5]);
      real q0 = E.q[qa + 3], q1 = E.q[qa + 4], q2 = E.q[qa + 5], q3 = E.q[qa + 6];
      real nrm = m_sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
      real in = RL(1.0) / nrm;
      real w0 = q0 * in;
      f3 vv = mk3(q1 * in, q2 * in, q3 * in);
      // d/dquat = (1/|q|) J(qhat)^T tau,  J = 2 [-v | w I + [v]x]
      E.qb[qa + 3] -= in * (-RL(2.0) * dot3(vv, tr));
      f3 gv = scl3(sub3(scl3(tr, w0), cross3(vv, tr)), RL(2.0) * in);
      E.qb[qa + 4] -= gv.x; E.qb[qa + 5] -= gv.y; E.qb[qa + 6] -= gv.z;
    } else {
      E.qb[jr.qa] -= E.dPq[jr.va];
    }
  }
  wsync();
  SIM_PHASE(E, PH_A_STATE);
}

// Adjoint of one substep from its pre-state alone: the forward linearisation is
// recomputed first (plain path, and the last substep of a recomputed segment).
template <int NV, class L>
__device__ __forceinline__ void substep_adjoint(const Scal* __restrict__ m, L& E,
                                                const JointRegs& jr, const ContactRegs& cr, int ln) {
  Chol C;
  int fb;
  substep_forward<NV>(m, E, jr, cr, ln, C, false, fb);
  substep_adjoint_core<NV>(m, E, jr, cr, ln, C, fb);
}

// --------------------------------------------------------------- linearisation tape
// Everything the adjoint of a substep reads from its forward pass, kept so that the
// reverse sweep does not recompute it: the pre-substep state, per frame the world screw S, velocity v, bias
// acceleration and spatial inertia, per contact sphere the force, contact point, its
// velocity and the depth, qdd, the post-substep velocities, the Cholesky rows, the
// reciprocal pivots and the FP64-fallback flag (the FP64 factor itself is not kept: a
// flagged substep is recomputed).  These fields are one contiguous block of EnvLDS, so
// a tape entry is a byte copy of it: 16 bytes per lane and instruction.

// make the post-substep state current (the in-place end of substep_forward)
template <class L>
__device__ __forceinline__ void commit_substep(const Scal* __restrict__ m, L& E, int ln) {
  if (ln < m->nq) E.q[ln] = E.qn[ln];
  if (ln < m->nv) E.qd[ln] = E.qdn[ln];
  if constexpr (L::kMtu > 0)
    for (int i = ln; i < m->n_mtu; i += SIM_WAVE) E.act[i] = E.actn[i];
  wsync();
  SIM_PHASE(E, PH_COMMIT);
}

// The block's fields sit where sim_tape_layout says (the host builds the word maps from it).
template <class L>
__device__ __forceinline__ constexpr bool tape_layout_ok() {
  constexpr SimTapeLayout T = sim_tape_layout(L::kJ, L::kV, L::kC);
  constexpr size_t r = sizeof(real);
  return offsetof(L, qd) == T.qd * r && offsetof(L, S) == T.S * r && offsetof(L, v) == T.v * r &&
         offsetof(L, ab) == T.ab * r && offsetof(L, Ib) == T.Ib * r && offsetof(L, cf) == T.cf * r &&
         offsetof(L, cx) == T.cx * r && offsetof(L, cvel) == T.cvel * r && offsetof(L, cdep) == T.cdep * r &&
         offsetof(L, qdd) == T.qdd * r && offsetof(L, qdn) == T.qdn * r && offsetof(L, M) == T.M * r &&
         offsetof(L, tdinv) == T.tdinv * r && offsetof(L, tfb) == T.tfb * r && offsetof(L, R) == T.R * r &&
         offsetof(L, p) == T.p * r && (L::kMtu == 0 || offsetof(L, act) == T.act * r);
}

typedef unsigned int tape_u32x4 __attribute__((ext_vector_type(4)));

// An entry (tape or factor cache) moves in 16-byte chunks of the LDS block: chunk w of the entry
// is the block's chunk off[w] (16-byte units from the block's start), and lane ln of the
// environment moves chunks ln, ln + LN, ... (consecutive lanes, consecutive 16 bytes).  A lane
// reads its chunks' block offsets once per kernel into registers; -1 past the entry's end.
template <int NCH>
struct ChunkMap {
  int off[NCH];
};
template <int NCH>
struct ChunkRegs {
  tape_u32x4 v[NCH];
};
template <int NCH, int LN>
__device__ __forceinline__ ChunkMap<NCH> chunk_map(const unsigned short* __restrict__ off, int nw, int ln) {
  ChunkMap<NCH> T;
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    const int w = i * LN + ln;
    T.off[i] = (w < nw) ? (int)off[w] : -1;
  }
  return T;
}
// streaming (non-temporal) stores and loads: entries must not displace the policy weights in L2
template <int NCH, int LN>
__device__ __forceinline__ void chunks_store(const ChunkMap<NCH>& T, const real* blk, real* __restrict__ dst, int ln) {
  const tape_u32x4* b = reinterpret_cast<const tape_u32x4*>(blk);
  tape_u32x4* d = reinterpret_cast<tape_u32x4*>(dst);
#pragma unroll
  for (int i = 0; i < NCH; ++i)
    if (T.off[i] >= 0) __builtin_nontemporal_store(b[T.off[i]], &d[i * LN + ln]);
}
template <int NCH, int LN>
__device__ __forceinline__ void chunks_prefetch(const ChunkMap<NCH>& T, ChunkRegs<NCH>& P, const real* __restrict__ src,
                                                int ln) {
  const tape_u32x4* s = reinterpret_cast<const tape_u32x4*>(src);
#pragma unroll
  for (int i = 0; i < NCH; ++i)
    if (T.off[i] >= 0) P.v[i] = __builtin_nontemporal_load(&s[i * LN + ln]);
}
template <int NCH>
__device__ __forceinline__ void chunks_restore(const ChunkMap<NCH>& T, real* blk, const ChunkRegs<NCH>& P) {
  tape_u32x4* b = reinterpret_cast<tape_u32x4*>(blk);
#pragma unroll
  for (int i = 0; i < NCH; ++i)
    if (T.off[i] >= 0) b[T.off[i]] = P.v[i];
}

template <class L>
using TapeMap = ChunkMap<L::kTapeChunksPerLane>;
template <class L>
using TapeRegs = ChunkRegs<L::kTapeChunksPerLane>;
template <class L>
__device__ __forceinline__ TapeMap<L> tape_map(const Scal* __restrict__ m, int ln) {
  return chunk_map<L::kTapeChunksPerLane, L::kLanes>(m->tab->tape_off, m->tape_nw, ln);
}

// the reciprocal pivots and the fallback flag into the block (both entries carry them)
template <int NV, class L>
__device__ __forceinline__ void stash_pivots(L& E, const Chol& C, int fb, int ln) {
  real dv = RL(0.0);
#pragma unroll
  for (int k = 0; k < NV; ++k) dv = (ln == k) ? C.dinv[k] : dv;
  if (ln < L::kV) {
    E.tdinv[ln] = dv;
    E.tfb[ln] = fb ? RL(1.0) : RL(0.0);
  }
  wsync();
}

// The factor into registers from the block: the model's nv rows of the factor (lower
// triangle) and pivots; a kernel compiled for NV > nv pads the matrix with the identity, whose
// factor is the identity (pivots 1), as the forward's factorisation left it.
template <int NV, class L>
__device__ __forceinline__ void factor_from_block(const Scal* __restrict__ m, const L& E, Chol& C, int& fb, int ln) {
  const int nv = m->nv;
  const int lr = ln < nv ? ln : 0;
  if (nv == NV) {
    // no padding: the lanes past the matrix read row 0 and are never read by the solves
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      C.row[k] = E.M[lr][k];
      C.col[k] = E.M[k][lr];
      C.dinv[k] = E.tdinv[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const real pad = (ln == k) ? RL(1.0) : RL(0.0);
      C.row[k] = (ln < nv && k < nv) ? E.M[lr][k] : pad;
      C.col[k] = (ln < nv && k < nv) ? E.M[k][lr] : pad;
      C.dinv[k] = (k < nv) ? E.tdinv[k] : RL(1.0);
    }
  }
  // uniform over the environment's lanes (its own LDS); over the wavefront only with 64 lanes
  if constexpr (L::kLanes == SIM_WAVE) fb = __builtin_amdgcn_readfirstlane(E.tfb[0] != RL(0.0) ? 1 : 0);
  else fb = (E.tfb[0] != RL(0.0)) ? 1 : 0;
}

// the new velocities as the forward computed them (qdn = qd + dt qdd)
template <class L>
__device__ __forceinline__ void rebuild_qdn(const Scal* __restrict__ m, L& E, int ln) {
  if (ln < m->nv) {
    const real dt = m->dt_sub;
    real qdn = E.qd[ln] + dt * E.qdd[ln];
    E.qdn[ln] = qdn;
  }
  wsync();
}

template <int NV, class L>
__device__ __forceinline__ void tape_store(const TapeMap<L>& T, L& E, const Chol& C, int fb, int ln,
                                           real* __restrict__ tp) {
  static_assert(offsetof(L, q) == 0, "tape block first");
  static_assert(tape_layout_ok<L>(), "LDS block as sim_tape_layout describes it");
  stash_pivots<NV>(E, C, fb, ln);
  chunks_store<L::kTapeChunksPerLane, L::kLanes>(T, &E.q[0], tp, ln);
  SIM_PHASE(E, PH_TAPE_STORE);
}

// A tape entry held in registers (the lane's chunks): the adjoint loads the next entry while
// the current substep's reverse runs, so the load latency is hidden.
template <class L>
__device__ __forceinline__ void tape_prefetch(const TapeMap<L>& T, TapeRegs<L>& P, const real* __restrict__ tp,
                                              int ln) {
  chunks_prefetch<L::kTapeChunksPerLane, L::kLanes>(T, P, tp, ln);
}

// tape_load from a prefetched entry: the chunks back into the block, the new velocities
// rebuilt, the factor into registers
template <int NV, class L>
__device__ __forceinline__ void tape_load_regs(const Scal* __restrict__ m, const TapeMap<L>& T, L& E, Chol& C,
                                               int& fb, int ln, const TapeRegs<L>& P) {
  // LDS ordering only (one wavefront per environment): the tape stores still in flight
  // need not complete here, and the registers wait for their own loads
  wsync();   // earlier LDS reads of the block complete before it is overwritten
  chunks_restore<L::kTapeChunksPerLane>(T, &E.q[0], P);
  wsync();
  rebuild_qdn(m, E, ln);
  factor_from_block<NV>(m, E, C, fb, ln);
  SIM_PHASE(E, PH_TAPE_LOAD);
}

// ---- factor cache (persistent path): the forward keeps every substep's Cholesky factor,
// reciprocal pivots and fallback flag (an entry of chunks of the block) and its accelerations
// qdd (a row of nv values); the adjoint rebuilds the states of a checkpoint segment from the
// accelerations and recomputes only the kinematics, contacts and inertias of each substep.
template <class L>
using FcMap = ChunkMap<L::kFcChunksPerLane>;
template <class L>
struct FcRegs {
  ChunkRegs<L::kFcChunksPerLane> c;
  real qdd, q, qd;   // lane ln: qdd[ln], and q[ln], qd[ln] of the pre-substep state
};
template <class L>
__device__ __forceinline__ FcMap<L> fc_map(const Scal* __restrict__ m, int ln) {
  return chunk_map<L::kFcChunksPerLane, L::kLanes>(m->tab->fc_off, m->fc_nw, ln);
}

template <int NV, class L>
__device__ __forceinline__ void fc_store(const Scal* __restrict__ m, const FcMap<L>& T, L& E, const Chol& C, int fb,
                                         int ln, real* __restrict__ entry, real* __restrict__ qrow) {
  stash_pivots<NV>(E, C, fb, ln);
  chunks_store<L::kFcChunksPerLane, L::kLanes>(T, &E.q[0], entry, ln);
  if (ln < m->nv) qrow[ln] = E.qdd[ln];
  SIM_PHASE(E, PH_TAPE_STORE);
}

// the entry, the accelerations and the pre-substep state [q | qd] (at most one coordinate and
// one velocity per lane: torque models, nq and nv at most the environment's lanes) into registers
template <class L>
__device__ __forceinline__ void fc_prefetch(const Scal* __restrict__ m, const FcMap<L>& T, FcRegs<L>& P,
                                            const real* __restrict__ entry, const real* __restrict__ qrow,
                                            const real* __restrict__ pre, int ln) {
  chunks_prefetch<L::kFcChunksPerLane, L::kLanes>(T, P.c, entry, ln);
  P.qdd = (ln < m->nv) ? qrow[ln] : RL(0.0);
  P.q = (ln < m->nq) ? pre[ln] : RL(0.0);
  P.qd = (ln < m->nv) ? pre[m->nq + ln] : RL(0.0);
}

// the entry and the accelerations only (the pre-substep state is filled in later)
template <class L>
__device__ __forceinline__ void fc_prefetch_entry(const Scal* __restrict__ m, const FcMap<L>& T, FcRegs<L>& P,
                                                  const real* __restrict__ entry, const real* __restrict__ qrow, int ln) {
  chunks_prefetch<L::kFcChunksPerLane, L::kLanes>(T, P.c, entry, ln);
  P.qdd = (ln < m->nv) ? qrow[ln] : RL(0.0);
}

// a prefetched entry back: the pre-substep state, factor and pivots into the block, qdd and
// the new velocities, and the substep's fallback flag (the factor enters registers later, with
// factor_from_block, so that it is not live across the kinematics recomputation)
template <class L>
__device__ __forceinline__ void fc_load_regs(const Scal* __restrict__ m, const FcMap<L>& T, L& E, int& fb, int ln,
                                             const FcRegs<L>& P) {
  wsync();
  chunks_restore<L::kFcChunksPerLane>(T, &E.q[0], P.c);
  if (ln < m->nq) E.q[ln] = P.q;
  if (ln < m->nv) {
    E.qd[ln] = P.qd;
    E.qdd[ln] = P.qdd;
  }
  wsync();
  rebuild_qdn(m, E, ln);
  // uniform over the environment's lanes (its own LDS); over the wavefront only with 64 lanes
  if constexpr (L::kLanes == SIM_WAVE) fb = __builtin_amdgcn_readfirstlane(E.tfb[0] != RL(0.0) ? 1 : 0);
  else fb = (E.tfb[0] != RL(0.0)) ? 1 : 0;
  SIM_PHASE(E, PH_TAPE_LOAD);
}

// the substep's accelerations (lane ln: qdd[ln]) from the cache, then the post-substep state
// made current (the state recursion of the forward, without its dynamics)
template <class L>
__device__ __forceinline__ void fc_step_state(const Scal* __restrict__ m, L& E, const JointRegs& jr, real qdd,
                                              int ln) {
  if (ln < m->nv) E.qdd[ln] = qdd;
  wsync();
  rebuild_qdn(m, E, ln);
  integrate_positions(m, E, jr, ln);
  wsync();
  if (ln < m->nq) E.q[ln] = E.qn[ln];
  if (ln < m->nv) E.qd[ln] = E.qdn[ln];
  wsync();
}
