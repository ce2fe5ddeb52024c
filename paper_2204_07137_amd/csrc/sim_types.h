// Types shared by the host ABI code and the device code: model tables, MLP and window
// kernel arguments, each templated on the arithmetic type of the path (float or double).
#pragma once
#include <stddef.h>
#include <stdint.h>

#define SIM_WAVE 64
#define SIM_MAXJ 32      // joint frames
#define SIM_MAXV 32      // velocity DOFs (one row of M per lane)
#define SIM_MAXQ 33      // position coordinates
#define SIM_MAXC 32      // contact spheres
#define SIM_MAXA 32      // actions of torque-driven models
#define SIM_MAXAM 160    // actions of muscle-driven models (motors + muscle excitations)
#define SIM_MAXMTU 160   // muscle-tendon units
#define SIM_MAXMPT 6     // path points per muscle-tendon unit
#define SIM_MAXOBS 288   // observation width
#define SIM_MAXHID 512   // MLP width
#define SIM_MAXL 4       // MLP linear layers
#define SIM_MAXTS 32     // steps of the scheduled subtree sums (a 32-frame chain needs 31)
#define SIM_MAXPAIR 576  // (frame, ancestor-or-self) pairs of the mass matrix, 9 rounds of 64 lanes
// linearisation tape of one substep: SIM_TAPE_REALS values (pre-substep state, frame
// screws, velocities, bias accelerations and inertias, contact data, accelerations, new
// velocities, the Cholesky rows, pivots and flag), plus the frame transforms and the
// activations for muscle models, padded to whole 1 KB blocks
#define SIM_TAPE_REALS 2465
// The compact per-environment LDS layout of small torque-driven models (CartPole, Ant): every
// table sized for at most SIM_C* entries, about a third of the full layout, so that more
// environments share a CU and several can share one wavefront (lanes per env 16, 32 or 64).
#define SIM_CJ 16        // joint frames
#define SIM_CV 16        // velocity DOFs (position coordinates: SIM_CV + 1)
#define SIM_CC 16        // contact spheres
#define SIM_CA 16        // actions
#define SIM_COBS 64      // observation width
#define SIM_CHID 128     // MLP width
#define SIM_CPAIR 64     // mass-matrix pairs
// reals of the linearisation tape block of a layout for J frames, V DOFs and C contacts:
// q, qd, S / v / ab / Ib per frame, force / point / velocity / depth per contact, qdd, qdn,
// the mass-matrix rows (V x (V + 1)), reciprocal pivots and the fallback flag
constexpr int sim_tape_reals(int J, int V, int C) {
  return (V + 1) + V + 28 * J + 10 * C + 2 * V + V * (V + 1) + 2 * V;
}
static_assert(sim_tape_reals(32, 32, 32) == SIM_TAPE_REALS, "tape block of the full layout");
// Offsets (in reals from the block's start) of the fields of the linearisation block of a
// layout with capacities J frames, V DOFs, C contacts, in their order in LDS: the state before
// the substep, per frame the screw, velocity, bias acceleration and spatial inertia, per contact
// the force, point, velocity and depth, the accelerations, new velocities, mass-matrix rows
// (then the Cholesky rows), reciprocal pivots, fallback flag, frame rotations and positions
// and the muscle activations.
struct SimTapeLayout { int q, qd, S, v, ab, Ib, cf, cx, cvel, cdep, qdd, qdn, M, tdinv, tfb, R, p, act; };
constexpr SimTapeLayout sim_tape_layout(int J, int V, int C) {
  return SimTapeLayout{0, V + 1, 2 * V + 1, 2 * V + 1 + 6 * J, 2 * V + 1 + 12 * J, 2 * V + 1 + 18 * J,
                       2 * V + 1 + 28 * J, 2 * V + 1 + 28 * J + 3 * C, 2 * V + 1 + 28 * J + 6 * C,
                       2 * V + 1 + 28 * J + 9 * C, 2 * V + 1 + 28 * J + 10 * C, 3 * V + 1 + 28 * J + 10 * C,
                       4 * V + 1 + 28 * J + 10 * C, 4 * V + 1 + 28 * J + 10 * C + V * (V + 1),
                       5 * V + 1 + 28 * J + 10 * C + V * (V + 1), 6 * V + 1 + 28 * J + 10 * C + V * (V + 1),
                       6 * V + 1 + 37 * J + 10 * C + V * (V + 1), 6 * V + 1 + 40 * J + 10 * C + V * (V + 1)};
}
// The tape entry of a substep holds only the fields the reverse reads, for the model's own
// sizes: q (nq), qd (nv), S / v / ab / Ib of its J frames, the nc contacts' data, qdd, the lower
// triangle of the Cholesky factor row by row, the reciprocal pivots and the flag (muscle models
// also R, p and the activations).  It moves in 16-byte chunks of the block: chunk w of an entry
// is the block's chunk tape_off[w] (in 16-byte units), and the list holds every chunk that
// contains one of those words.  A run of n words covers at most ceil(n / words-per-chunk) + 1
// chunks, so an entry never needs more than sim_tape_chunk_cap chunks.
constexpr int sim_tape_chunk_cap(int J, int V, int C, int nmtu, int elem) {
  return (((V + 1) + V + 28 * J + 10 * C + V + V * (V + 1) / 2 + V + 1 + (nmtu > 0 ? 12 * J + nmtu : 0)) * elem + 15) / 16 +
         2 * (V + 16);
}
// A factor-cache entry: the lower triangle of the Cholesky factor row by row, the reciprocal
// pivots and the fallback flag, in 16-byte chunks of the block (fc_off, as tape_off).
constexpr int sim_fc_chunk_cap(int V, int elem) { return ((V * (V + 1) / 2 + V + 1) * elem + 15) / 16 + 2 * (V + 2); }
#define SIM_MAXFCW 384
// the factor cache's adjoint holds a checkpoint segment's accelerations in registers: k <= 16
#define SIM_FC_MAXK 16
#define SIM_MAXTAPEW 2432   // capacity of the chunk list (the largest layout in FP64 needs 1305)
// BF16 tile bytes of one layer's forward or input-adjoint operand set
static inline size_t sim_bf16_tiles_bytes(int n_rows, int n_k) {
  return (size_t)((n_rows + 15) / 16) * ((n_k + 31) / 32) * 64 * 8 * 2;
}

enum { J_FREE = 0, J_HINGE = 1, J_SLIDE = 2 };
enum { TASK_NONE = 0, TASK_CARTPOLE = 1, TASK_ANT = 2, TASK_HUMANOID = 3, TASK_MTU = 4 };

template <typename T>
struct DevModelT {
  int J, nq, nv, na, nc, ns, od, task, floating, has_last_action, substeps, max_depth;
  int n_mtu, n_motor, nck;   // muscles; motors (the first n_motor actions); nq + nv + n_mtu
  int term;                  // early termination below term_h (root height)
  T dt_sub, g, kn, kd, kt, mu, klim;
  T chol_thr;   // FP64 refactorisation when the smallest pivot <= chol_thr * largest diagonal
  T tau_act, fl_w, vmax;     // activation time constant, force-length width, max fibre speed (l_opt/s)
  T term_h;
  int parent[SIM_MAXJ], jtype[SIM_MAXJ], qadr[SIM_MAXJ], vadr[SIM_MAXJ], depth[SIM_MAXJ];
  int first_child[SIM_MAXJ], next_sib[SIM_MAXJ], act_of_joint[SIM_MAXJ], limited[SIM_MAXJ];
  // schedule of the forward subtree sums: at step s lane group g adds frame j into its parent p,
  // ts_edge[g][s] = j | p << 5 | 1 << 10 (0: nothing); ts_steps steps
  unsigned short ts_edge[4][SIM_MAXTS];
  int ts_steps;
  T offset[SIM_MAXJ * 3], axis[SIM_MAXJ * 3], mass[SIM_MAXJ], com[SIM_MAXJ * 3];
  T inertia[SIM_MAXJ * 6];   // xx yy zz xy xz yz about the COM, frame axes
  T lower[SIM_MAXJ], upper[SIM_MAXJ], gear[SIM_MAXJ];
  T armature[SIM_MAXV];
  int cbody[SIM_MAXC];
  T cpos[SIM_MAXC * 3], crad[SIM_MAXC];
  unsigned int cmask[SIM_MAXJ];   // bit c set when contact c belongs to frame j
  // mass-matrix entries M[va_k][va_i] for every non-root frame i and every k in its
  // ancestors-or-self: packed i | k << 5 | va_i << 10 | va_k << 15 | (k is FREE) << 20 | 1 << 21
  int npair;
  int pair[SIM_MAXPAIR];
  // the packed linearisation tape: 16-byte chunks per entry and the block offset of every
  // chunk, in 16-byte units
  int tape_nw;
  unsigned short tape_off[SIM_MAXTAPEW];
  // the factor-cache entry: chunks per entry and their block offsets (16-byte units)
  int fc_nw;
  unsigned short fc_off[SIM_MAXFCW];
  // muscle-tendon units, point-major so that lanes (one unit each) read contiguously
  int mtu_npt[SIM_MAXMTU];
  int mtu_body[SIM_MAXMPT * SIM_MAXMTU];     // [point][unit]
  T mtu_pos[SIM_MAXMPT * 3 * SIM_MAXMTU];    // [point][xyz][unit], in the body frame
  T mtu_fmax[SIM_MAXMTU], mtu_lopt[SIM_MAXMTU], mtu_lslack[SIM_MAXMTU];
  // the same tables packed for one vector load per point and one per unit (what the kernels
  // read): [point][unit][x, y, z, body] and [unit][F_max, l_opt, l_slack, points]
  T mtu_pt[SIM_MAXMPT * SIM_MAXMTU * 4] __attribute__((aligned(32)));
  T mtu_par[SIM_MAXMTU * 4] __attribute__((aligned(32)));
};

template <typename T>
struct MlpArgsT {
  int nl;                      // linear layers
  int bf16;                    // layers on the BF16 matrix cores (FP32 accumulation)
  int dims[SIM_MAXL + 1];
  // BF16 tiles of 64 lanes x 8 values, one matrix-core operand each (workspace):
  const uint16_t* Pf[SIM_MAXL];   // forward: [ceil(out/16)][ceil(in/32)] tiles of W
  const uint16_t* Pb[SIM_MAXL];   // input adjoint: [ceil(in/16)][ceil(out/32)] tiles of W^T
  const T* W[SIM_MAXL];        // [out][pad64(in)] zero-padded copy (workspace)
  const T* WT[SIM_MAXL];       // [in][pad64(out)] zero-padded copy (workspace)
  const T* b[SIM_MAXL];        // [out] (caller)
  const T* src[SIM_MAXL];      // [out][in] caller weights, copied by the prep kernel
  // layer normalisation of every hidden layer's ELU output (App. A.2), or none (ln = 0):
  // y = g (e - mean(e)) / sqrt(var(e) + ln_eps) + beta over the layer's outputs
  int ln;
  T ln_eps;
  const T* lng[SIM_MAXL];      // [out] gain of hidden layer l (caller)
  const T* lnb[SIM_MAXL];      // [out] bias of hidden layer l (caller)
};

// blocks of the policy-gradient pass's layer-normalisation adjoint (fixed: their partial sums
// are reduced in block order, so the result does not depend on the row count)
#define SIM_LN_BLOCKS 256

// phases of the window kernels' profile (a build with -DSIM_PHASE_PROFILE; ids in sim_math.h)
#define SIM_NPHASE 40

template <typename T>
struct WinArgsT {
  const DevModelT<T>* model;
  int N, h, k, closed_loop;
  T gamma, scale;
  const T* s0;
  const T* actions_in;
  const T* noise;   // [h][N][na] standard normal draws of the stochastic policy, or null
  const T* log_std; // [na] log of the policy's standard deviation (with noise)
  MlpArgsT<T> actor, critic;
  T* s_h;
  T* obs;
  T* actions;
  T* rewards;
  T* value;
  uint8_t* nonfinite;
  int* fallback;    // [N] substeps whose factorisation fell back to FP64 (optional)
  int* adhesive;    // [N] contact evaluations (substep x contact) with a pulling normal force (optional)
  T* ckpt;          // [n_ckpt][N][nq+nv] (persistent and plain paths)
  T* adj;           // [N][nq+nv+na] adjoint carried between plain launches
  T* tape;          // tape_full: [h*S][N] tape entries written by the forward; else the
                    // adjoint's segment tape [N][k-1] entries, tape_ws reals apart
  int tape_full;
  int tape_ws;      // reals between consecutive tape entries (the packed words, rounded up)
  // factor cache (persistent path, optional): fc [h*S][N] entries fc_ws reals apart, fcq
  // [h*S][N][nv] accelerations; the adjoint keeps a segment's pre-substep states in tape
  // ([N][k][nck])
  T* fc;
  T* fcq;
  int fc_ws;
  const T* obs_in;
  const T* actions_fw;
  const T* s_h_in;
  const T* grad_s_h;
  T* dL_da;
  T* dL_ds0;
  // early termination: reset states [N][ns]; done flags [h][N] (workspace, and the optional
  // output); seg [h+1][N]: the first frame of the discount segment that frame t belongs to
  // (row h: the segment that the terminal value closes)
  const T* reset;
  uint8_t* done_out;
  uint8_t* done_ws;
  int* seg_ws;
  // observation normalisation: the networks see (o - obs_mean) * obs_inv_std (both [od]) or o
  const T* obs_mean;
  const T* obs_inv_std;
  // the actor's hidden activations of every frame, [h][N][hid_w] (workspace, closed loop):
  // written by the forward, read by the adjoint's input VJP
  T* hid;
  int hid_w;
  // the window's loss: per env [N] and the sum over envs [1] (forward, optional)
  T* loss_env;
  T* loss;
  // phase-profile build only: [SIM_NPHASE] shader-clock cycle totals over all environments
  unsigned long long* prof;
};

// Several models' windows in one launch (mixed-morphology batch): work-table slot s covers
// blocks [start[s], start[s+1]) with the window arguments A[s] of a model with nv[s] DOFs.
#define SIM_MAXGROUP 6
template <typename T>
struct GroupArgsT {
  int n;
  int start[SIM_MAXGROUP + 1];   // first block of each slot (a block holds 64 / lanes envs)
  int nv[SIM_MAXGROUP];
  int mtu[SIM_MAXGROUP];      // slot's model has muscles
  int lanes[SIM_MAXGROUP];    // 0: full layout, one env per wavefront; 16 / 32 / 64: compact layout
  WinArgsT<T> A[SIM_MAXGROUP];
};

// Policy-parameter gradient pass over the rows (frame, env) of one window.
template <typename T>
struct ThetaArgsT {
  int M;                      // rows: h * N
  int nl;                     // linear layers of the actor
  int dims[SIM_MAXL + 1];
  int splits;                 // row chunks of the weight-gradient reductions
  const T* W[SIM_MAXL];       // [out][in] caller weights
  const T* b[SIM_MAXL];
  const T* x0;                // [M][dims[0]] observations o_0 .. o_{h-1}
  const T* x_shift;           // [dims[0]] or null: the first layer reads (x0 - x_shift) * x_scale
  const T* x_scale;
  const T* act;               // [M][na] actions
  const T* da;                // [M][na] dL/da
  int mtu;                    // muscle task: actions u = (tanh(y) + 1) / 2, else a = tanh(y)
  const T* noise;             // [M][na] draws of the stochastic policy, or null
  const T* log_std;           // [na]
  T* out_log_std;             // [na] dL/dlog_std (with noise), or null
  T* H[SIM_MAXL];             // H[l] (l >= 1): [M][dims[l]] hidden activations
  long ldH[SIM_MAXL];         // row stride of H[l] (0: dims[l])
  int hidden_given;           // H holds the activations already (the window's own): no recompute
  T* d0;                      // [M][max dim] layer adjoints (ping-pong)
  T* d1;
  T* part;                    // [splits][max out*(in+1)] partial weight gradients
  T* out;                     // flat dL/dtheta: W_0, b_0, W_1, b_1, ...
  long off_w[SIM_MAXL], off_b[SIM_MAXL];
  // layer normalisation of the hidden layers: H[l] then holds the ELU outputs, st + r * ldst
  // the per-row mean and inverse deviation of each hidden layer (the window's, or computed by
  // the hidden-layer pass with ln_eps), Y[l] ([M][dims[l]], scratch) the normalised layer
  // inputs, lnpart ([ln_blocks][2][max width]) the per-block partial sums of the gain and bias
  // gradients (flat at off_g / off_beta)
  int ln;
  T ln_eps;
  const T* lng[SIM_MAXL];
  const T* lnb[SIM_MAXL];
  T* st;
  long ldst;
  T* Y[SIM_MAXL];
  T* lnpart;
  int ln_blocks;
  long off_g[SIM_MAXL], off_beta[SIM_MAXL];
};

// Adam over a list of parameter tensors whose gradient and moments are flat, in list order.
#define SIM_MAX_TENSORS 16
template <typename T>
struct LearnAdamT {
  int n;
  T* p[SIM_MAX_TENSORS];
  long size[SIM_MAX_TENSORS];
  const T* g;
  T* m;
  T* v;
  T lr, b1, b2, eps, bc1, bc2;   // bc = 1 - beta^step (bias corrections)
};

// Critic fit over shuffled minibatches (the layer gradients run through G, whose x0 / M are
// set per minibatch and whose out is the flat gradient buffer).
template <typename T>
struct CriticFitT {
  ThetaArgsT<T> G;      // layer-gradient pass
  const T* obs;         // [rows][obs_dim]
  const T* obs_mean;    // [obs_dim] or null: rows are gathered as (obs - obs_mean) * obs_inv_std
  const T* obs_inv_std;
  const T* targets;     // [rows]
  const int* perm;      // [n_iter][rows]
  int rows, n_iter, n_mb;
  T* x;                 // [rows][obs_dim] gathered minibatch
  T* y;                 // [rows]
  T* vbuf;              // [rows] critic outputs
  T* W[SIM_MAXL];       // critic weights, updated in place
  T* bvec[SIM_MAXL];
  T* lng[SIM_MAXL];     // with layer normalisation: the hidden layers' gains and biases, updated
  T* lnb[SIM_MAXL];     // in place (G.lng / G.lnb view the same arrays)
  T* m;                 // flat Adam moments
  T* v;
  int adam_step;        // Adam steps taken before the call
  T lr, b1, b2, eps;
  T* loss_out;          // [n_iter * n_mb] minibatch losses before each step (optional)
};

// Launchers implemented once per arithmetic type (kernels_f32.hip, kernels_f64.hip).
#define SIM_DECLARE_LAUNCHERS(NS, T)                                                        \
  namespace NS {                                                                            \
  int launch_forward(const WinArgsT<T>& A, int plain, int substeps, int nv, int mtu, int lanes, void* stream); \
  int launch_adjoint(const WinArgsT<T>& A, int plain, int substeps, int nv, int mtu, int lanes, void* stream); \
  int launch_prep_weights(const T* W, T* WT, T* Wp, int n_out, int n_in, void* stream);   \
  int launch_prep_bf16(const T* W, uint16_t* Pf, uint16_t* Pb, int n_out, int n_in, void* stream); \
  int launch_theta(const ThetaArgsT<T>& A, void* stream);                                  \
  int launch_group(const GroupArgsT<T>& G, int adjoint, int mtu, size_t lds_bytes, void* stream); \
  size_t group_lds_bytes(int lanes, int mtu);                                              \
  int prepare_group(size_t lds_bytes);                                                     \
  }
SIM_DECLARE_LAUNCHERS(sim_f32, float)
SIM_DECLARE_LAUNCHERS(sim_f64, double)
// the learning-episode update (learn.hip)
#define SIM_DECLARE_LEARN(NS, T)                                                           \
  namespace NS {                                                                           \
  int launch_adam(const LearnAdamT<T>& A, void* stream);                                   \
  int launch_soft_update(T* t, const T* o, long n, T alpha, void* stream);                 \
  int launch_td_lambda(const T* r, const T* v, const uint8_t* d, int h, int N, T g, T l, T* out, void* s); \
  int launch_critic_values(const ThetaArgsT<T>& A, T* out, void* stream);                  \
  int launch_obs_stats(const T* x, long rows, int od, double count, T* mean, T* var, T* inv_std, double eps,   \
                       void* stream);                                                      \
  int launch_critic_fit(const CriticFitT<T>& F, void* stream);                             \
  }
SIM_DECLARE_LEARN(sim_l32, float)
SIM_DECLARE_LEARN(sim_l64, double)
