// Device math for one arithmetic type.  Included inside a namespace with `real` defined
// as float or double (kernels_f32.hip, kernels_f64.hip).
//
// Spatial vectors are 6-vectors in world-aligned Plücker coordinates whose reference
// point O is the root position of the current substep (the world origin for fixed-base
// models): motion (w, v_O), force (n_O, f).

#define RL(x) static_cast<real>(x)

typedef DevModelT<real> DevModel;
typedef MlpArgsT<real> MlpArgs;
typedef WinArgsT<real> WinArgs;
typedef GroupArgsT<real> GroupArgs;

// Uniform model scalars, copied once per kernel into registers (the tables in global
// memory are read only at kernel start).
struct Scal {
  int J, nq, nv, na, nc, ns, od, task, floating, has_last_action, substeps, max_depth, ts_steps, term;
  int n_mtu, n_motor, nck;
  int tape_nw;           // 16-byte chunks of a packed tape entry
  int fc_nw;             // 16-byte chunks of a factor-cache entry
  real dt_sub, g, kn, kd, kt, mu, klim, chol_thr;
  real tau_act, fl_w, vmax, term_h;
  const DevModel* tab;   // the model's tables (muscle paths) in global memory
};
__device__ __forceinline__ Scal load_scal(const DevModel* __restrict__ m) {
  Scal s;
  s.J = m->J; s.nq = m->nq; s.nv = m->nv; s.na = m->na; s.nc = m->nc; s.ns = m->ns; s.od = m->od;
  s.task = m->task; s.floating = m->floating; s.has_last_action = m->has_last_action;
  s.substeps = m->substeps; s.max_depth = m->max_depth; s.ts_steps = m->ts_steps;
  s.dt_sub = m->dt_sub; s.g = m->g; s.kn = m->kn; s.kd = m->kd; s.kt = m->kt; s.mu = m->mu; s.klim = m->klim;
  s.chol_thr = m->chol_thr;
  s.n_mtu = m->n_mtu; s.n_motor = m->n_motor; s.nck = m->nck;
  s.tau_act = m->tau_act; s.fl_w = m->fl_w; s.vmax = m->vmax;
  s.term = m->term; s.term_h = m->term_h;
  s.tape_nw = m->tape_nw;
  s.fc_nw = m->fc_nw;
  s.tab = m;
  return s;
}

__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
// reciprocal square root: hardware v_rsq in FP32 (about 1 ulp), exact division in FP64
__device__ __forceinline__ float m_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double m_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ void m_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void m_sincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ float m_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double m_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_tanh(float x) { return tanhf(x); }
__device__ __forceinline__ double m_tanh(double x) { return tanh(x); }
__device__ __forceinline__ float m_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double m_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float m_fabs(float x) { return fabsf(x); }
__device__ __forceinline__ double m_fabs(double x) { return fabs(x); }
__device__ __forceinline__ float m_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double m_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float m_fmin(float x, float y) { return fminf(x, y); }
__device__ __forceinline__ double m_fmin(double x, double y) { return fmin(x, y); }
__device__ __forceinline__ float m_fmax(float x, float y) { return fmaxf(x, y); }
__device__ __forceinline__ double m_fmax(double x, double y) { return fmax(x, y); }
__device__ __forceinline__ bool m_isfinite(float x) { return isfinite(x); }
__device__ __forceinline__ bool m_isfinite(double x) { return isfinite(x); }

// broadcast lane l's value (l uniform)
__device__ __forceinline__ float rdl(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double rdl(double x, int l) {
  long long v = __builtin_bit_cast(long long, x);
  int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Orders the LDS accesses of the environment's lanes.  A workgroup here is one wavefront,
// and one wavefront's LDS operations are performed in program order, so a value written
// by one lane is seen by a later read of another lane without waiting for the write; the
// fences only keep the compiler from moving memory accesses across this point.  (Direct
// global-to-LDS transfers are not LDS operations in this sense and keep a full barrier.)
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- phase profile.  A build with -DSIM_PHASE_PROFILE accumulates, per environment, the
// shader-clock cycles (s_memtime) from one mark to the next under the id of the later mark, in
// the environment's LDS, and adds the totals to a device table when the window ends; in the
// product build the marks are empty.  A mark names the phase that ends at it.
enum {
  PH_FRAME_BEGIN = 0,   // observation, actor, reward, action store (frame start)
  PH_F_FK = 1,          // joint rotations and frame transforms (pointer jumping)
  PH_F_VEL = 2,         // motion subspaces, velocities, bias accelerations
  PH_F_CONTACT = 3,     // contact forces
  PH_F_MUSCLE = 4,      // muscle wrenches
  PH_F_NE = 5,          // body inertias, Newton-Euler forces, joint torques
  PH_F_TREESUM = 6,     // subtree sums of forces and composite inertias
  PH_F_BIAS = 7,        // bias into the right-hand side, CRBA columns, root block
  PH_F_CRBA = 8,        // mass-matrix entries
  PH_F_CHOL = 9,        // Cholesky factorisation (with the row load and the pivot test)
  PH_F_FACTOR = 10,     // factor rows to LDS and columns back (or the FP64 fallback)
  PH_F_SOLVE = 11,      // the two triangular solves and the velocity update
  PH_F_INTEG = 12,      // positions (and activations), in-place commit
  PH_TAPE_STORE = 13,   // a tape entry to HBM
  PH_COMMIT = 14,       // post-substep state made current
  PH_CKPT = 15,         // checkpoint store / load
  PH_A_SEED = 16,       // terminal critic seed
  PH_A_INTEG = 17,      // integrator reverse
  PH_A_LAMBDA = 18,     // lambda = M^-1 qdd_bar
  PH_A_PATH = 19,       // accelerations and virtual velocities along the root paths
  PH_A_CONTACT = 20,    // contact adjoints
  PH_A_MUSCLE = 21,     // muscle adjoints
  PH_A_BODY = 22,       // per-body terms
  PH_A_TREESUM = 23,    // subtree sums of the seven spatial vectors
  PH_A_DERIV = 24,      // closed-form derivatives per joint
  PH_A_STATE = 25,      // adjoint of the pre-substep state
  PH_TAPE_LOAD = 26,    // a prefetched entry back into LDS and the factor into registers
  PH_TAPE_PREFETCH = 27,// issuing the next entry's loads
  PH_A_FRAME = 28,      // frame-level reverse (reward, actor input VJP, observation)
  PH_WINDOW_END = 29,   // terminal observation, critic, outputs
  PH_TERM = 30,         // early-termination test and reset
  PH_FC_STATES = 31,   // factor cache: a segment's pre-substep states from the cached accelerations
  PH_FM_PATH = 32,     // forward muscles: path geometry and tensions (per pass of 64 units)
  PH_FM_ACC = 33,      // forward muscles: point forces into the per-body wrench table
  PH_AM_PATH = 34,     // muscle adjoint: path geometry and tensions recomputed
  PH_AM_DERIV = 35,    // muscle adjoint: virtual velocities, tension and direction derivatives
  PH_AM_ACC = 36,      // muscle adjoint: per-body terms into the three tables
  PH_FB_OBS = 37,      // frame start: observation and its store
  PH_FB_MLP = 38,      // frame start: the actor MLP and the hidden activations' store
  PH_AF_MLP = 39       // frame-level reverse: the actor's input VJP with its operand loads
};
static_assert(PH_AF_MLP < SIM_NPHASE, "phase ids within the profile table");
#ifdef SIM_PHASE_PROFILE
template <int LN>
__device__ __forceinline__ void phase_mark(unsigned long long* P, int id);
#define SIM_PHASE(E, id) phase_mark<L::kLanes>((E).prof, (id))
#else
#define SIM_PHASE(E, id) ((void)0)
#endif

// lane src's value, src chosen per lane (a wavefront-wide permute through the LDS
// crossbar: no LDS memory, no barrier); every lane of the wavefront must be active
__device__ __forceinline__ int pull(int x, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, x); }
__device__ __forceinline__ float pull(float x, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double pull(double x, int src) {
  long long v = __builtin_bit_cast(long long, x);
  int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(v & 0xffffffffll));
  int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(v >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---- one environment on LN lanes of a wavefront (LN = 16, 32 or 64; an environment's lanes
// are contiguous and aligned).  With LN = 64 these are the plain wavefront operations.
template <int LN>
__device__ __forceinline__ int grp_base() { return LN == SIM_WAVE ? 0 : ((int)threadIdx.x & (SIM_WAVE - LN)); }
template <int LN>
__device__ __forceinline__ int grp_lane() { return LN == SIM_WAVE ? (int)threadIdx.x : ((int)threadIdx.x & (LN - 1)); }
#ifdef SIM_PHASE_PROFILE
template <int LN>
__device__ __forceinline__ void phase_mark(unsigned long long* P, int id) {
  const unsigned long long now = __builtin_amdgcn_s_memtime();
  if (grp_lane<LN>() == 0) {
    P[id] += now - P[SIM_NPHASE];
    P[SIM_NPHASE] = now;
  }
}
template <int LN>
__device__ __forceinline__ void phase_start(unsigned long long* P) {
  if (grp_lane<LN>() == 0) {
    for (int i = 0; i < SIM_NPHASE; ++i) P[i] = 0ull;
    P[SIM_NPHASE] = __builtin_amdgcn_s_memtime();
  }
}
template <int LN>
__device__ __forceinline__ void phase_flush(const unsigned long long* P, unsigned long long* out) {
  if (out && grp_lane<LN>() == 0)
    for (int i = 0; i < SIM_NPHASE; ++i) atomicAdd(&out[i], P[i]);
}
#endif

// the value of the environment's lane k (k the same on all lanes of the environment)
template <int LN, class T>
__device__ __forceinline__ T bcast(T x, int k) {
  if constexpr (LN == SIM_WAVE) return rdl(x, k);
  else return pull(x, grp_base<LN>() + k);
}
// the value of the environment's lane src (src chosen per lane); every lane must be active
template <int LN, class T>
__device__ __forceinline__ T pull_g(T x, int src) {
  return pull(x, grp_base<LN>() + src);
}
// bits of the environment's lanes in a wavefront ballot
template <int LN>
__device__ __forceinline__ unsigned long long grp_ballot(bool p) {
  const unsigned long long b = __ballot(p);
  if constexpr (LN == SIM_WAVE) return b;
  else return (b >> grp_base<LN>()) & ((1ull << LN) - 1ull);
}
template <int LN>
__device__ __forceinline__ bool grp_all(bool p) {
  if constexpr (LN == SIM_WAVE) return __all(p);
  else return grp_ballot<LN>(!p) == 0ull;
}

// ------------------------------------------------------------------ small vector math
struct f3 { real x, y, z; };
__device__ __forceinline__ f3 mk3(real a, real b, real c) { f3 r; r.x = a; r.y = b; r.z = c; return r; }
__device__ __forceinline__ f3 add3(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 sub3(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 scl3(f3 a, real s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ real dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
  return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ f3 ld3(const real* p) { return mk3(p[0], p[1], p[2]); }
__device__ __forceinline__ void st3(real* p, f3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

// 3x3 row-major matrix times vector
__device__ __forceinline__ f3 mv3(const real* R, f3 v) {
  return mk3(R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
             R[6] * v.x + R[7] * v.y + R[8] * v.z);
}
__device__ __forceinline__ f3 mtv3(const real* R, f3 v) {
  return mk3(R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
             R[2] * v.x + R[5] * v.y + R[8] * v.z);
}

// spatial 6-vectors as (angular, linear) pairs
struct sv { f3 a, l; };
__device__ __forceinline__ sv mksv(f3 a, f3 l) { sv r; r.a = a; r.l = l; return r; }
__device__ __forceinline__ sv zsv() { return mksv(mk3(0, 0, 0), mk3(0, 0, 0)); }
__device__ __forceinline__ sv addsv(sv a, sv b) { return mksv(add3(a.a, b.a), add3(a.l, b.l)); }
__device__ __forceinline__ sv subsv(sv a, sv b) { return mksv(sub3(a.a, b.a), sub3(a.l, b.l)); }
__device__ __forceinline__ sv sclsv(sv a, real s) { return mksv(scl3(a.a, s), scl3(a.l, s)); }
__device__ __forceinline__ real dotsv(sv m, sv f) { return dot3(m.a, f.a) + dot3(m.l, f.l); }
__device__ __forceinline__ sv ldsv(const real* p) { return mksv(mk3(p[0], p[1], p[2]), mk3(p[3], p[4], p[5])); }
__device__ __forceinline__ void stsv(real* p, sv a) {
  p[0] = a.a.x; p[1] = a.a.y; p[2] = a.a.z; p[3] = a.l.x; p[4] = a.l.y; p[5] = a.l.z;
}
// motion x motion
__device__ __forceinline__ sv crm(sv a, sv b) {
  return mksv(cross3(a.a, b.a), add3(cross3(a.a, b.l), cross3(a.l, b.a)));
}
// motion x* force
__device__ __forceinline__ sv crf(sv a, sv f) {
  return mksv(add3(cross3(a.a, f.a), cross3(a.l, f.l)), cross3(a.a, f.l));
}
// spatial force of the 3-force g applied at point x
__device__ __forceinline__ sv spf(f3 x, f3 g) { return mksv(cross3(x, g), g); }
// velocity of the point x under the motion m
__device__ __forceinline__ f3 ptv(sv m, f3 x) { return add3(m.l, cross3(m.a, x)); }

// spatial inertia in 10 numbers: m, h = m c (3), Ibar = rotational inertia about O (xx yy zz xy xz yz)
__device__ __forceinline__ sv iapply(const real* I, sv v) {
  real m = I[0];
  f3 h = mk3(I[1], I[2], I[3]);
  f3 w = v.a;
  f3 Iw = mk3(I[4] * w.x + I[7] * w.y + I[8] * w.z, I[7] * w.x + I[5] * w.y + I[9] * w.z,
              I[8] * w.x + I[9] * w.y + I[6] * w.z);
  return mksv(add3(Iw, cross3(h, v.l)), add3(scl3(v.l, m), cross3(w, h)));
}

// max over the environment's LN lanes (butterfly)
template <int LN>
__device__ __forceinline__ real grp_max(real x) {
#pragma unroll
  for (int off = LN / 2; off >= 1; off >>= 1) x = m_fmax(x, __shfl_xor(x, off, SIM_WAVE));
  return x;
}

// wave-wide sum (deterministic butterfly over 64 lanes)
__device__ __forceinline__ real wave_sum(real x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, SIM_WAVE);
  return x;
}
