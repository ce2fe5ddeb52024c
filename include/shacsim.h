/*
 * shacsim — batched differentiable articulated-body windows on one AMD Instinct GPU.
 *
 * C ABI of the hot path of Short-Horizon Actor-Critic (Xu et al., ICLR 2022): N
 * independent environments are simulated forward over a window of h frames by the
 * simulator map s_{t+1} = F(s_t, a_t) (Sec. 3.1), with the actions produced in the
 * loop by a deterministic MLP policy (Sec. 3.3) or given open loop, and the window is
 * then differentiated backward (Sec. 3.1 Eq. "backward"; App. A.1) to give the
 * gradients of the short-horizon actor loss (Sec. 3.3 Eq. "policy_loss")
 *     L = -1/(N h) sum_i [ sum_t gamma^t R(s_t, a_t) + gamma^h V(s_h) ]
 * with respect to the actions and the window's initial states.  Gradients stop at the
 * window start (Sec. 3.3: gradients are cut between learning episodes).
 *
 * Dynamics (Sec. 3.1 Eq. "fwd_dynamics"): generalized coordinates, RNEA bias forces,
 * CRBA mass matrix, a per-environment dense Cholesky solve, penalty ground contact with
 * the linear-step Coulomb friction law (Sec. 3.1 contact equation), joint-limit
 * penalties (Sec. 3.1 limit equation) and semi-implicit Euler with S substeps per frame.
 *
 * Conventions
 *   - Every array passed to sim_forward_window / sim_adjoint_window is a DEVICE pointer
 *     owned by the caller, row-major and env-major:  X[t][env][component].  Real arrays
 *     are float32 when the handle's precision is SIM_PREC_FP32 (the production path:
 *     dynamics, policy and critic in FP32) and float64 when it is SIM_PREC_FP64 (the
 *     same kernels instantiated in double precision, for verification at scale).
 *   - State  s = [q (nq) | qd (nv) | a_prev (na, tasks whose observation holds the last
 *     action)].  A free root has q = (x, y, z, qw, qx, qy, qz) and qd = (world velocity of
 *     the root origin, world angular velocity).
 *   - MLP weights are W[out][in] and b[out] per linear layer (ELU hidden layers, linear
 *     output; the policy output is squashed by tanh).
 *   - The calls enqueue work on the given HIP stream and return; they allocate nothing
 *     (the caller passes a workspace of sim_workspace_bytes()) and may be captured in a
 *     HIP graph.  The forward and the adjoint of one window must use the same handle,
 *     workspace and stream order.
 * Errors
 *   - Functions return a SimStatus.  Argument errors are detected before anything is
 *     enqueued and leave the outputs untouched; sim_last_error() then describes the
 *     problem (per calling thread).  Numerical failure of one environment is data, not an
 *     error: its nonfinite flag is set and the other environments are unaffected.
 */
#ifndef SHACSIM_H
#define SHACSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SIM_OK = 0,
  SIM_E_ARG = -1,         /* bad argument: null pointer, size, shape or option */
  SIM_E_HANDLE = -2,      /* null or destroyed handle */
  SIM_E_HIP = -3,         /* a HIP runtime call failed */
  SIM_E_MODEL = -4,       /* model description invalid or beyond the compiled limits */
  SIM_E_WORKSPACE = -5,   /* workspace missing or smaller than sim_workspace_bytes() */
  SIM_E_UNSUPPORTED = -6  /* valid request this build does not implement */
} SimStatus;

enum { SIM_JOINT_FREE = 0, SIM_JOINT_HINGE = 1, SIM_JOINT_SLIDE = 2 };
enum { SIM_TASK_NONE = 0, SIM_TASK_CARTPOLE = 1, SIM_TASK_ANT = 2, SIM_TASK_HUMANOID = 3, SIM_TASK_MTU = 4 };
enum { SIM_PATH_PERSISTENT = 0, SIM_PATH_PLAIN = 1, SIM_PATH_TAPE = 2 };
enum { SIM_PREC_FP32 = 0, SIM_PREC_FP64 = 1 };
enum { SIM_MLP_FP32 = 0, SIM_MLP_BF16 = 1 };

/* Compiled limits. */
#define SIM_MAX_JOINTS 32
#define SIM_MAX_DOFS 32
#define SIM_MAX_CONTACTS 32
#define SIM_MAX_ACTIONS 32             /* motors */
#define SIM_MAX_MTU 160                /* muscle-tendon units */
#define SIM_MAX_MTU_POINTS 6           /* path points per unit */
#define SIM_MAX_MUSCLE_ACTIONS 160     /* motors + muscles of a muscle model */
#define SIM_MAX_OBS 288
#define SIM_MAX_HIDDEN 512
#define SIM_MAX_LAYERS 4

/* Articulated model (host memory, read during sim_create only).  Frame j hangs from frame
 * parent[j] (-1 = world, parents listed first) at offset[j] (parent frame, no fixed
 * rotation), then moves through its joint (FREE root, HINGE about axis[j], SLIDE along
 * axis[j]).  mass/com/inertia describe the body rigidly attached to frame j (inertia about
 * the COM in frame axes, 3x3 row-major; mass 0 = massless frame).  Actuator i drives
 * joint act_joint[i] with torque/force gear[i] * a_i.  Contact spheres (body, centre in
 * the body frame, radius) touch the ground plane z = 0. */
typedef struct SimModelDesc {
  int n_joints;
  const int* parent;
  const int* jtype;
  const double* offset;          /* [J][3] */
  const double* axis;            /* [J][3], unit */
  const double* mass;            /* [J] */
  const double* com;             /* [J][3] */
  const double* inertia;         /* [J][3][3] */
  const int* limited;            /* [J] */
  const double* lower;           /* [J] */
  const double* upper;           /* [J] */
  int n_act;
  const int* act_joint;          /* [n_act] */
  const double* gear;            /* [n_act] */
  const double* armature;        /* [nv] added to the mass-matrix diagonal */
  int n_contacts;
  const int* contact_body;       /* [C] */
  const double* contact_pos;     /* [C][3] */
  const double* contact_radius;  /* [C] */
  double gravity;                /* m/s^2, along -z */
  double kn, kd, kt, mu;         /* contact stiffness, damping, friction stiffness, Coulomb mu */
  double klim;                   /* joint-limit stiffness */
  double dt;                     /* frame duration (s) */
  int substeps;                  /* S: semi-implicit Euler substeps per frame */
  int task;                      /* SIM_TASK_*: observation and reward definition */
  int has_last_action;           /* state carries the previous action */
  /* Muscle-tendon units (Sec. 3.1: muscle actuation through attachment sites on several
   * bodies; Hill-type reading).  Unit i is a polyline through mtu_npt[i] points, point k
   * fixed at mtu_pos[i][k] in frame mtu_body[i][k].  With path length L and rate Ldot,
   * rigid tendon l_m = L - l_slack, the tension is
   *   F = max(0, F_max act exp(-((l_m/l_opt - 1)/fl_width)^2) (1 + Ldot/(vmax l_opt)))
   * pulling every path point towards its neighbours; the activation follows
   * act' = act + dt (u - act)/tau_act per substep with the excitation u.  The actions
   * are [motor actions (n_act) | excitations (n_mtu)], the state gains the n_mtu
   * activations after q, qd (and a_prev). */
  int n_mtu;                     /* 0 = torque-driven model */
  const int* mtu_npt;            /* [n_mtu], 2..SIM_MAX_MTU_POINTS */
  const int* mtu_body;           /* [n_mtu][SIM_MAX_MTU_POINTS] */
  const double* mtu_pos;         /* [n_mtu][SIM_MAX_MTU_POINTS][3] */
  const double* mtu_fmax;        /* [n_mtu] N */
  const double* mtu_lopt;        /* [n_mtu] m */
  const double* mtu_lslack;      /* [n_mtu] m */
  double tau_act;                /* s */
  double fl_width;
  double vmax;                   /* optimal fibre lengths per second */
  /* Early termination (App. A.3: a task ends when the root falls below a height): with
   * term_enabled, an env whose free root is below term_height (m, world z) at the end of a
   * frame is marked done, replaced by its reset state (SimForwardIO.reset_states), and its
   * discount restarts; the reset cuts the gradient (the reset state is a constant).  Needs a
   * FREE root; runs on the persistent and tape paths. */
  int term_enabled;
  double term_height;
} SimModelDesc;

typedef struct SimOptions {
  int n_envs;                    /* N */
  int horizon;                   /* h frames per window */
  int ckpt_interval;             /* k: the forward stores the state every k substeps (k | S);
                                    1 for the tape and plain paths */
  int path;                      /* SIM_PATH_PERSISTENT: one launch per window, the adjoint
                                      recomputes each k-substep segment from its checkpoint;
                                    SIM_PATH_TAPE: one launch per window, the forward also
                                      records every substep's linearisation (Cholesky factor,
                                      frame screws, inertias, contacts; about 9.5 KB per substep
                                      and env in FP32) and the adjoint recomputes nothing (k = 1);
                                    SIM_PATH_PLAIN: one launch per frame start and per substep,
                                      the state of every substep goes through HBM (k = 1) */
  int closed_loop;               /* 1: actions from the actor MLP; 0: actions given */
  int actor_layers;              /* linear layers of the actor (closed loop) */
  int actor_dims[SIM_MAX_LAYERS + 1];
  int critic_layers;             /* linear layers of the critic (terminal value) */
  int critic_dims[SIM_MAX_LAYERS + 1];
  double gamma;                  /* discount */
  int precision;                 /* SIM_PREC_FP32 or SIM_PREC_FP64 (arithmetic and I/O type) */
  double chol_fp64_threshold;    /* FP32 path: an environment's mass matrix is refactorised in
                                    FP64 for a substep whose smallest Cholesky pivot is <= this
                                    times its largest diagonal entry, or not finite (1e-6 is the
                                    documented default; a value > 1 forces FP64 every substep) */
  int policy_grad;               /* closed loop: 1 = the workspace also holds the scratch of the
                                    policy-parameter gradient, and sim_adjoint_window accepts
                                    dL_dtheta */
  int mlp_precision;             /* SIM_MLP_FP32, or SIM_MLP_BF16 (FP32 path only): actor and
                                    critic layers on the BF16 matrix cores with BF16 weights and
                                    layer inputs and FP32 accumulation, biases and activations;
                                    their input adjoints likewise (the output adjoint in BF16).
                                    The dynamics stay FP32. */
  int lanes_per_env;             /* 0: the full per-environment layout, one environment per 64-lane
                                    wavefront (every model); 16, 32 or 64: the compact layout of
                                    small torque-driven models (at most 16 frames, 16 DOFs, 16
                                    contacts, 16 actions, 64 observations, MLP widths <= 128 and
                                    <= 8 x lanes, 64 mass-matrix pairs, frames / DOFs / contacts
                                    / coordinates <= lanes), 64 / lanes environments per
                                    wavefront and several wavefronts per CU; n_envs must then be a
                                    multiple of 64 / lanes.  FP32 path, FP32 MLPs, persistent or
                                    tape path.  Results are bitwise those of the full layout. */
  int factor_cache;              /* persistent path, torque-driven models: 1 = the forward also
                                    keeps every substep's Cholesky factor, reciprocal pivots and
                                    accelerations qdd (the factorisation cached for the backward
                                    pass, Sec. 3.1; about 1.6 KB per substep and env for the
                                    27-DOF humanoid in FP32), and the adjoint rebuilds each
                                    checkpoint segment's states from the accelerations and
                                    recomputes only the kinematics, contacts and body inertias of
                                    each substep (no mass matrix, factorisation or solve).
                                    0 = the adjoint recomputes whole substeps from the
                                    checkpoints.  Results are bitwise the same either way.
                                    Needs ckpt_interval <= 16. */
  int layer_norm;                /* 1: every hidden layer of the actor and of the critic is followed
                                    by a layer normalisation of its ELU outputs, y = g (e - mean)
                                    / sqrt(var + 1e-5) + beta over the layer's outputs (App. A.2);
                                    the gains and biases are window inputs (actor_ln_* /
                                    critic_ln_*), and dL_dtheta then holds their gradients after
                                    each hidden layer's W, b.  FP32 / FP64 MLPs.  The critic calls
                                    take the critic's gains and biases too (sim_critic_values_ln,
                                    SimCriticFitIO.critic_ln_*; sim_critic_values and
                                    sim_critic_values_noalloc refuse such a handle).  0: no
                                    normalisation (the benchmark configurations). */
} SimOptions;

typedef struct SimHandle SimHandle;

typedef struct SimForwardIO {
  const void* s0;                           /* [N][ns] */
  const void* actions_in;                   /* [h][N][na], open loop only */
  const void* actor_w[SIM_MAX_LAYERS];      /* closed loop only: W [out][in] */
  const void* actor_b[SIM_MAX_LAYERS];      /* b [out] */
  const void* critic_w[SIM_MAX_LAYERS];
  const void* critic_b[SIM_MAX_LAYERS];
  const void* actor_ln_g[SIM_MAX_LAYERS];   /* with opt.layer_norm: per hidden layer l of the actor,
                                               its normalisation's gain [dims[l+1]] */
  const void* actor_ln_b[SIM_MAX_LAYERS];   /* and bias [dims[l+1]] (device; unused entries NULL) */
  const void* critic_ln_g[SIM_MAX_LAYERS];  /* the same for the critic */
  const void* critic_ln_b[SIM_MAX_LAYERS];
  void* workspace;                          /* sim_workspace_bytes() bytes, 256-byte aligned */
  size_t workspace_bytes;
  void* s_h;                                /* [N][ns] out: state after h frames */
  void* obs;                                /* [h+1][N][obs_dim] out */
  void* actions;                            /* [h][N][na] out */
  void* rewards;                            /* [h][N] out */
  void* value;                              /* [N] out: critic value of s_h */
  uint8_t* nonfinite;                       /* [N] out, optional: 1 if s_h is not finite */
  int32_t* fp64_refactor_count;             /* [N] out, optional: substeps refactorised in FP64 */
  /* Stochastic policy (Sec. 3.3: a_t ~ N(mu(s_t), sigma), sampled by reparameterisation):
   * with both set, the pre-squash policy output is y_t = mu(o_t) + exp(log_std) * eps_t and
   * the action squash(y_t); both null = the deterministic policy.  Closed loop only. */
  const void* noise;                        /* [h][N][na] standard normal draws eps, or NULL */
  const void* log_std;                      /* [na], or NULL */
  const void* reset_states;                 /* [N][ns] the states terminated envs restart from
                                               (required with term_enabled) */
  uint8_t* done;                            /* [h][N] out, optional: 1 if the env terminated at
                                               the end of frame t */
  /* Observation normalisation (Sec. 3.3, running mean and deviation): with both set, the
   * actor and the critic read (o - obs_mean) * obs_inv_std, both [obs_dim] (for example from
   * sim_obs_stats_update); both NULL = raw observations.  The obs output stays raw. */
  const void* obs_mean;
  const void* obs_inv_std;
  /* [N] out, optional: per env, the contact evaluations of the window (substeps x contacts)
   * that penetrate (d < 0) with a pulling normal force, i.e. where the literal damping term
   * of the contact model (Sec. 3.1) exceeds the stiffness term (d_dot > k_n / k_d). */
  int32_t* adhesive_count;
  /* The short-horizon actor loss (Sec. 3.3, Eq. "policy_loss"), optional outputs: loss_env [N]
   * each env's term -1/(N h) (sum_t gamma^(t - t0) r_t + gamma^(h - t0) V(o_h)), with t0 the
   * start of the env's discount segment (0 without early termination; no terminal value
   * after a termination in the last frame), and loss [1] their sum in a fixed order. */
  void* loss_env;
  void* loss;
} SimForwardIO;

typedef struct SimAdjointIO {
  const void* s0;                           /* as given to the forward */
  const void* actions;                      /* forward output */
  const void* obs;                          /* forward output */
  const void* s_h;                          /* forward output */
  const void* actor_w[SIM_MAX_LAYERS];
  const void* actor_b[SIM_MAX_LAYERS];
  const void* critic_w[SIM_MAX_LAYERS];
  const void* critic_b[SIM_MAX_LAYERS];
  const void* actor_ln_g[SIM_MAX_LAYERS];   /* as given to the forward (opt.layer_norm) */
  const void* actor_ln_b[SIM_MAX_LAYERS];
  const void* critic_ln_g[SIM_MAX_LAYERS];
  const void* critic_ln_b[SIM_MAX_LAYERS];
  void* workspace;                          /* written by the matching forward */
  size_t workspace_bytes;
  const void* grad_s_h;                     /* [N][ns] optional extra upstream dL/ds_h */
  double loss_scale;                        /* factor on the loss seeds: 1/(N h) for the actor loss
                                               of Sec. 3.3 (times dOut/dL when chained); 0 = only
                                               grad_s_h is propagated */
  void* dL_da;                              /* [h][N][na] out: partial dL/da_t (App. A.1) */
  void* dL_ds0;                             /* [N][ns] out: total dL/ds_0 (App. A.1) */
  void* dL_dtheta;                          /* optional out (needs opt.policy_grad): dL/dtheta of the
                                               actor (App. A.1), the sum over frames and envs of
                                               (d pi / d theta)^T dL/da_t, flat in layer order
                                               W_0 [out][in], b_0, W_1, b_1, ... (with
                                               opt.layer_norm each hidden layer's W, b are
                                               followed by its normalisation's gain and bias);
                                               bitwise reproducible for a given handle */
  const void* noise;                        /* as given to the forward (stochastic policy), or NULL */
  const void* log_std;                      /* as given to the forward, or NULL */
  void* dL_dlog_std;                        /* [na] optional out (with dL_dtheta and noise): the
                                               sum over frames and envs of dL/dy_t * exp(log_std)
                                               * eps_t; bitwise reproducible */
  const void* obs_mean;                     /* as given to the forward, or NULL */
  const void* obs_inv_std;
} SimAdjointIO;

/* Validates the model and options and uploads the constant tables to the current device.
 * Returns SIM_E_MODEL for a model beyond the compiled limits. */
int sim_create(const SimModelDesc* model, const SimOptions* opt, SimHandle** out);

/* Bytes of device workspace the caller must provide (checkpoint arena + MLP copies). */
size_t sim_workspace_bytes(const SimHandle* h);

/* Sizes derived from the model: state width, observation width, actions, nq, nv. */
int sim_dims(const SimHandle* h, int* n_state, int* n_obs, int* n_act, int* nq, int* nv);

/* Forward window: h frames of (observation, policy, reward, S substeps). */
int sim_forward_window(SimHandle* h, const SimForwardIO* io, void* hip_stream);

/* Reverse of the forward window: dL/da_t and dL/ds_0 of the actor loss and, when
 * dL_dtheta is given, the actor's parameter gradient (App. A.1).  The parameter gradient
 * takes the actor's hidden activations that the forward stored in the workspace for every
 * frame and env, carries the action adjoint back through the layers and contracts the layer
 * adjoints with the layer inputs over all h*N rows on the matrix cores.
 * The adjoint reads what the matching forward left in the workspace (checkpoints, tape,
 * hidden activations, termination flags): no other forward on the same handle and workspace
 * may run between a window's forward and its adjoint, or the gradients are those of the
 * other window.  Nothing here can detect that; the Python binding tags each forward and
 * refuses an adjoint of a stale one. */
int sim_adjoint_window(SimHandle* h, const SimAdjointIO* io, void* hip_stream);

void sim_destroy(SimHandle* h);

/* ---- Mixed-morphology batches.  A group runs the windows of several handles (models
 * with different DOF, contact and action counts, each with its own N, weights and
 * workspace) as ONE kernel launch: a work table maps every block to (model, env), the
 * models ordered by decreasing per-env cost so that the longest windows start first (the
 * environments of all models are independent, Sec. 3.1).  The launch (with the weight
 * preparation and, in the adjoint, the parameter-gradient passes) is captured once into a
 * HIP graph on a stream the group owns and replayed with hipGraphLaunch on the caller's
 * stream; it is captured again when the arguments change.  Results are bitwise those of
 * the members' own sim_forward_window / sim_adjoint_window calls. */
#define SIM_MAX_GROUP 6
typedef struct SimGroup SimGroup;

/* members: n (1..SIM_MAX_GROUP) distinct handles of one precision on the current device,
 * persistent or tape path.  cost_hint: optional per-env cost of each member (e.g. the
 * us_per_env of sim_tune) for the dispatch order; NULL = estimate from the model.  The
 * handles must outlive the group. */
int sim_group_create(SimHandle* const* members, int n, const double* cost_hint, SimGroup** out);
/* ios[i] is member i's argument block, as for its own call. */
int sim_group_forward(SimGroup* g, const SimForwardIO* ios, void* hip_stream);
int sim_group_adjoint(SimGroup* g, const SimAdjointIO* ios, void* hip_stream);
/* order[s] (optional) = member index dispatched in work-table slot s; n_captures
 * (optional) = graphs captured so far (a call with the same arguments as the previous
 * one of its kind replays its graph). */
int sim_group_info(const SimGroup* g, int* order, int* n_captures);
void sim_group_destroy(SimGroup* g);

/* ---- Autotuner.  Times forward + adjoint windows of one model on the caller's inputs
 * for every launch configuration whose workspace fits workspace_budget: the tape path and
 * the persistent path at every checkpoint interval k dividing S (for torque-driven models
 * and k <= 16 with and without the factor cache), each in the full layout and,
 * for small models whose n_envs allows it, in the compact layout with 64, 32 and 16 lanes per
 * environment (opt->lanes_per_env is ignored); returns the fastest (median of reps windows
 * after a warm-up).  opt supplies everything else (N, h, MLP
 * shapes, precision).  io supplies s0, the weights (or actions_in) and the forward output
 * buffers, which the tuner overwrites; its workspace fields are ignored.  A set-up call:
 * it allocates and frees its own workspaces and synchronizes the stream. */
typedef struct SimTuneResult {
  int path;                      /* SIM_PATH_TAPE or SIM_PATH_PERSISTENT */
  int ckpt_interval;             /* k for the chosen path */
  size_t workspace_bytes;        /* workspace of the chosen configuration */
  double ms_window;              /* its forward + adjoint time per window */
  int n_candidates;              /* configurations timed */
  int lanes_per_env;             /* the chosen layout (SimOptions.lanes_per_env) */
  int factor_cache;              /* the chosen SimOptions.factor_cache */
} SimTuneResult;
int sim_tune(const SimModelDesc* model, const SimOptions* opt, const SimForwardIO* io,
             size_t workspace_budget, int reps, void* hip_stream, SimTuneResult* out);

/* ---- Device ceilings (measurement probes, not part of a window).  The roofline of the
 * window kernels is quoted against AMD's published MI355X figures and against these
 * measured ones.
 * sim_probe_fma: times an FP32 FMA loop (eight independent chains per lane, no packed
 * instructions, 4096 x 256 threads) on the stream and returns the achieved FP32 VALU
 * TFLOP/s.  scratch: caller-owned device buffer of at least sim_probe_fma_bytes() bytes
 * (the loop's results are written there).  Synchronizes the stream.
 * sim_probe_copy: times a device-to-device copy of `bytes` (a multiple of 16; both device
 * pointers 16-byte aligned, caller-owned, not overlapping) and returns GB/s counting
 * bytes read plus bytes written.  Synchronizes the stream.  Both return SIM_E_ARG on bad
 * arguments before any launch and SIM_E_HIP on a failed launch. */
size_t sim_probe_fma_bytes(void);
int sim_probe_fma(void* scratch, size_t scratch_bytes, void* hip_stream, double* tflops);
int sim_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream, double* gbs);

/* ---- Learning-episode update (Sec. 3.3, Algorithm "SHAC" and Eqs. "critic_loss",
 * "td-lambda"; hyperparameters of App. A.2).  The calls that follow a window: one Adam step
 * of the policy on dL_dtheta, TD-lambda estimates of the window's states from the target
 * critic, the critic's mean-squared-error fit over shuffled minibatches with Adam, and the
 * smooth update of the target critic.  Pointers are device pointers unless stated;
 * `precision` (SIM_PREC_FP32 / SIM_PREC_FP64) is the element type of the float buffers.
 * Argument errors return SIM_E_ARG before any launch; failed launches SIM_E_HIP. */
#define SIM_MAX_TENSORS 16

/* Adam (Kingma and Ba) on n_tensors (<= SIM_MAX_TENSORS) parameter tensors: tensors and sizes
 * are host arrays (device pointers, element counts); grad, m and v are flat device arrays of
 * sum(sizes) elements in tensor order (for the actor: the layout of dL_dtheta, W_0, b_0, W_1,
 * b_1, ...); step is this step's 1-based index (bias correction); m and v are updated. */
int sim_adam_step(void* const* tensors, const size_t* sizes, int n_tensors, const void* grad, void* m,
                  void* v, int step, double lr, double beta1, double beta2, double eps, int precision,
                  void* hip_stream);

/* target_i <- alpha target_i + (1 - alpha) online_i, elementwise per tensor (host arrays of
 * device pointers and element counts). */
int sim_soft_update(void* const* target, const void* const* online, const size_t* sizes, int n_tensors,
                    double alpha, int precision, void* hip_stream);

/* TD-lambda estimates: rewards [h][N]; values [h+1][N], the target critic at the window's
 * states s_0 .. s_h (s_0's value is not used); done [h][N] (device, optional: the forward
 * window's termination flags), where a frame that ended in termination has the estimate r_t
 * (its returns stop there and the fallen state has no value); out targets [h][N]. */
int sim_td_lambda(const void* rewards, const void* values, const uint8_t* done, int h, int n_envs, double gamma,
                  double lambda, void* targets, int precision, void* hip_stream);

/* The critic calls use the handle's critic shape and precision and a caller-owned workspace
 * of at least sim_critic_workspace_bytes(h, rows) bytes (rows: the most rows of one call). */
size_t sim_critic_workspace_bytes(const SimHandle* h, int rows);

/* values [rows] = V(obs [rows][obs_dim]) with the given critic weights (host arrays of device
 * pointers, W [out][in], b [out]); with obs_mean and obs_inv_std ([obs_dim], both or neither)
 * the critic reads (obs - obs_mean) * obs_inv_std. */
int sim_critic_values(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                      const void* const* critic_b, const void* obs_mean, const void* obs_inv_std, void* values,
                      void* workspace, size_t workspace_bytes, void* hip_stream);

/* sim_critic_values for a handle with layer_norm (App. A.2: a layer normalisation after every
 * hidden layer's ELU): critic_ln_g / critic_ln_b are host arrays of device pointers to each
 * hidden layer's gain and bias [dims[l + 1]].  Each row's mean and variance are computed over
 * the layer's outputs (one wavefront per row, a fixed butterfly order).  Without layer_norm
 * the gains and biases are ignored and may be null. */
int sim_critic_values_ln(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                         const void* const* critic_b, const void* const* critic_ln_g,
                         const void* const* critic_ln_b, const void* obs_mean, const void* obs_inv_std,
                         void* values, void* workspace, size_t workspace_bytes, void* hip_stream);

typedef struct SimCriticFitIO {
  const void* obs;              /* [rows][obs_dim] states of the window (o_0 .. o_{h-1}) */
  const void* targets;          /* [rows] their TD-lambda estimates (treated as constants) */
  int rows;
  const int32_t* perm;          /* [n_iter][rows] permutations of 0 .. rows-1 (device) */
  int n_iter;                   /* passes over the rows */
  int n_minibatch;              /* minibatches per pass: rows [mb rows / n, (mb + 1) rows / n) of perm */
  void* critic_w[SIM_MAX_LAYERS];   /* the critic being fitted, updated in place */
  void* critic_b[SIM_MAX_LAYERS];
  void* adam_m;                 /* flat Adam moments of the critic (W_0, b_0, W_1, ...) */
  void* adam_v;
  int adam_step;                /* Adam steps taken before this call */
  double lr, beta1, beta2, eps;
  void* loss_out;               /* [n_iter * n_minibatch] optional: each minibatch's mean squared
                                   error before its step */
  void* workspace;
  size_t workspace_bytes;
  const void* obs_mean;         /* [obs_dim] optional (with obs_inv_std): the critic reads */
  const void* obs_inv_std;      /* (obs - obs_mean) * obs_inv_std */
  void* critic_ln_g[SIM_MAX_LAYERS];   /* with layer_norm: each hidden layer's normalisation gain */
  void* critic_ln_b[SIM_MAX_LAYERS];   /* and bias [dims[l + 1]], updated in place; adam_m / adam_v
                                          then hold W_0, b_0, g_0, beta_0, W_1, ... (the gain and
                                          bias of a hidden layer after its W, b).  Ignored
                                          without layer_norm. */
} SimCriticFitIO;

/* Running observation statistics (Sec. 3.3): merges rows [rows][dim] of observations (device)
 * into the running count, mean [dim] and population variance var [dim] of all observations
 * merged before (count = 0: mean and var are only written), and writes
 * inv_std [dim] = 1 / sqrt(var + eps).  The caller keeps the count: the new count is
 * count + rows.  Pairwise (Chan-Golub-LeVeque) update with FP64 sums in a fixed order. */
int sim_obs_stats_update(const void* obs, long rows, int dim, double count, void* mean, void* var, void* inv_std,
                         double eps, int precision, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sim_critic_values without a workspace.
 * The critic's hidden-layer activations live in a static device array of 64 MiB that the
 * library holds on every GPU it runs on until the process ends, so rows x (sum of the critic's
 * hidden widths) x element size must fit in 64 MiB (after 256-byte alignment of each layer's
 * block; the humanoid's 76-128-128-1 critic in FP32: 65536 rows), else SIM_E_WORKSPACE before
 * any launch.  Arguments, layouts and results as for sim_critic_values; nothing is allocated
 * or freed.  Every call on a GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and give wrong values; serialise them.  The array keeps the last
 * call's activations, which nothing reads. */
int sim_critic_values_noalloc(SimHandle* h, const void* obs, int rows, const void* const* critic_w,
                              const void* const* critic_b, const void* obs_mean, const void* obs_inv_std,
                              void* values, void* hip_stream);

/* Fits the critic: for every pass and minibatch, the mean of (V(o) - target)^2 over the
 * minibatch, its gradient through the critic's layers, one Adam step.  The order of the
 * reductions is fixed, so the result is bitwise reproducible. */
int sim_critic_fit(SimHandle* h, const SimCriticFitIO* io, void* hip_stream);

/* Description of the last error on the calling thread ("" if none). */
const char* sim_last_error(void);

/* ---- Layout of the ABI structures as this library was compiled, for bindings written in
 * other languages to check their own declarations against: for the structure `which`, its
 * size in bytes (field < 0) or the byte offset of its field-th member in declaration order
 * (0-based).  Returns (size_t)-1 for an unknown structure or member index.  Pure host code. */
enum { SIM_ABI_MODEL_DESC = 0, SIM_ABI_OPTIONS = 1, SIM_ABI_FORWARD_IO = 2, SIM_ABI_ADJOINT_IO = 3,
       SIM_ABI_TUNE_RESULT = 4, SIM_ABI_CRITIC_FIT_IO = 5 };
size_t sim_abi_layout(int which, int field);

/* ---- Phase profile of the window kernels (diagnostics, not part of the method).  A library
 * built with -DSIM_PHASE_PROFILE (python -m paper_2204_07137_amd.build --phase-profile, which
 * writes libshacsim_phase.so) accumulates the shader-clock cycles every environment spends in
 * each phase of the persistent and tape window kernels (kinematics, contacts, Cholesky, ...;
 * the ids are the PH_* constants of csrc/sim_math.h) into a per-device table of 40 totals.
 * This call synchronises the current device, copies the first n (0 <= n <= 40) totals to the
 * host array out and, if reset, clears the table.  Returns the number of phases (40), or
 * SIM_E_UNSUPPORTED from a product build (no table, no marks). */
int sim_phase_profile(unsigned long long* out, int n, int reset);

#ifdef __cplusplus
}
#endif
#endif /* SHACSIM_H */
