// Observations, rewards, the deterministic MLP policy / critic and their adjoints, one
// environment per wavefront.
//
// Observations and rewards follow the task definitions of App. A.3 (CartPole Swing Up,
// Ant, Humanoid); "up" and "heading" are the z-z and x-x entries of the root rotation.
// The MLP has ELU hidden layers and a linear output (App. A.2); the policy squashes its
// output with tanh.


// The library keeps two zero-padded copies of every weight matrix in its workspace:
// WT [in][out_pad] for the forward (each lane owns out_pad/64 consecutive outputs) and
// W [out][in_pad] for the input adjoint (each lane owns in_pad/64 consecutive inputs),
// pad = next multiple of 64, so that the inner loops have a compile-time block size and
// unconditional, coalesced vector loads.
__host__ __device__ __forceinline__ int pad64(int n) { return (n + SIM_WAVE - 1) / SIM_WAVE * SIM_WAVE; }

// ---------------------------------------------------------------- BF16 matrix-core layers
// One environment's layer is a matrix-vector product.  It runs on the 16x16x32 BF16
// matrix instruction with the layer input as row 0 of the A operand (the other rows are
// zero) and 16 outputs as the columns of B, accumulating in FP32; lanes 0..15 then hold
// the 16 outputs of the tile.  Weights are pre-packed so that every B operand is one
// coalesced 1 KB load: lane l of a tile holds W[o0 + l % 16][k0 + 8 (l / 16) + j], j < 8.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite values)
__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// LDS x (n values) -> LDS BF16 operand, zero-padded to a multiple of 32
__device__ __forceinline__ void to_bf16(const real* x, uint16_t* xb, int n, int ln) {
  const int np = (n + 31) / 32 * 32;
  for (int i = ln; i < np; i += SIM_WAVE) xb[i] = (i < n) ? f2bf((float)x[i]) : (uint16_t)0;
  wsync();
}

// out[r] (r < nr) = sum_k Wt[r][k] xb[k] over nk inputs, Wt in tiles of P; with the bias,
// the ELU for hidden forward layers, or the ELU' factor from hin for the input adjoint.
__device__ __forceinline__ void mlp_tiles_bf16(const uint16_t* __restrict__ P, const uint16_t* xb, int nk,
                                               int nr, int ln, const real* bias, bool elu,
                                               const real* hin, real* dst) {
  const int nkt = (nk + 31) / 32, nrt = (nr + 15) / 16;
  const int lk = ln >> 4;
  for (int t0 = 0; t0 < nrt; t0 += 4) {
    f32x4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the weight tiles of two k-steps (up to eight) are requested before the first product,
    // so the loop waits for one memory latency per two k-steps, not per tile; the products
    // accumulate in k order as before
    int kt = 0;
    for (; kt + 2 <= nkt; kt += 2) {
      bf16x8 b[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          b[q][u] = (t0 + u < nrt) ? *reinterpret_cast<const bf16x8*>(P + ((size_t)((t0 + u) * nkt + kt + q) * SIM_WAVE + ln) * 8)
                                   : bf16x8{};
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8 a = *reinterpret_cast<const bf16x8*>(xb + (kt + q) * 32 + lk * 8);
        if (ln & 15) a = bf16x8{};
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t0 + u < nrt) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][u], acc[u], 0, 0, 0);
      }
    }
    for (; kt < nkt; ++kt) {
      bf16x8 a = *reinterpret_cast<const bf16x8*>(xb + kt * 32 + lk * 8);
      if (ln & 15) a = bf16x8{};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (t0 + u < nrt) {
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(P + ((size_t)((t0 + u) * nkt + kt) * SIM_WAVE + ln) * 8);
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[u], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = (t0 + u) * 16 + ln;
      if (ln < 16 && r < nr) {
        real z = (real)acc[u][0];
        if (bias) {
          z += bias[r];
          if (elu && z <= RL(0.0)) z = m_expm1(z);
        } else if (hin) {
          const real hv = hin[r];
          z *= (hv > RL(0.0)) ? RL(1.0) : (hv + RL(1.0));
        }
        dst[r] = z;
      }
    }
  }
}

__device__ __forceinline__ void mlp_forward_bf16(const MlpArgs& P, const real* x, real* h0, real* h1,
                                                 real* out, uint16_t* xb, int ln) {
  const real* in = x;
  for (int l = 0; l < P.nl; ++l) {
    const int ni = P.dims[l], no = P.dims[l + 1];
    real* dst = (l == P.nl - 1) ? out : ((l & 1) ? h1 : h0);
    to_bf16(in, xb, ni, ln);
    mlp_tiles_bf16(P.Pf[l], xb, ni, no, ln, P.b[l], l < P.nl - 1, nullptr, dst);
    wsync();
    in = dst;
  }
}

__device__ __forceinline__ void mlp_vjp_input_bf16(const MlpArgs& P, const real* h0, const real* h1,
                                                   real* gout, real* gbuf, real* xbar, uint16_t* xb, int ln) {
  const real* g = gout;
  for (int l = P.nl - 1; l >= 0; --l) {
    const int ni = P.dims[l], no = P.dims[l + 1];
    real* dst = (l == 0) ? xbar : gbuf;
    to_bf16(g, xb, no, ln);          // g is not read again: dst may alias it
    const real* hin = (l >= 1) ? (((l - 1) & 1) ? h1 : h0) : nullptr;
    mlp_tiles_bf16(P.Pb[l], xb, no, ni, ln, nullptr, false, hin, dst);
    wsync();
    g = dst;
  }
}

// NCH consecutive weights of one lane as one vector load where the width allows
// (16 or 8 bytes, aligned because rows are padded to 64 * NCH values).
template <int NCH>
__device__ __forceinline__ void load_lane_block(const real* __restrict__ p, real* w) {
  if constexpr (NCH == 4 && sizeof(real) == 4) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const v4*>(p);
    w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3];
  } else if constexpr (NCH == 2) {
    typedef real v2 __attribute__((ext_vector_type(2)));
    const v2 v = *reinterpret_cast<const v2*>(p);
    w[0] = v[0]; w[1] = v[1];
  } else {
#pragma unroll
    for (int c = 0; c < NCH; ++c) w[c] = p[c];
  }
}

// Weight rows are requested MLP_BATCH at a time, all before the first is used: the compiler
// otherwise waits for each row's load before requesting the next (the kernels use every
// register), paying one memory latency per row.  The FMA order is that of a row-by-row loop.
#define MLP_BATCH 8

// Each of the environment's LN lanes owns NCH consecutive outputs (rows padded to a multiple
// of 64 = NCH * LN), so a weight row is one coalesced vector load per lane.
template <int NCH, int LN>
__device__ __forceinline__ void mlp_layer_fwd(const real* __restrict__ WT, const real* __restrict__ bb,
                                              const real* in, real* dst, int ni, int no, bool hidden, int ln) {
  const int nop = NCH * LN;
  real acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int o = ln * NCH + c;
    acc[c] = (o < no) ? bb[o] : RL(0.0);
  }
  const real* base = WT + ln * NCH;
  int i = 0;
  for (; i + MLP_BATCH <= ni; i += MLP_BATCH) {
    real w[MLP_BATCH][NCH];
#pragma unroll
    for (int u = 0; u < MLP_BATCH; ++u) load_lane_block<NCH>(base + (size_t)(i + u) * nop, w[u]);
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < MLP_BATCH; ++u) {
      const real xi = in[i + u];
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] = m_fma(w[u][c], xi, acc[c]);
    }
  }
  for (; i < ni; ++i) {
    const real xi = in[i];
    real w[NCH];
    load_lane_block<NCH>(base + (size_t)i * nop, w);
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = m_fma(w[c], xi, acc[c]);
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int o = ln * NCH + c;
    if (o < no) {
      real z = acc[c];
      dst[o] = (hidden && z <= RL(0.0)) ? m_expm1(z) : z;
    }
  }
}

// input adjoint of one layer: lane owns NCH consecutive inputs
template <int NCH, int LN>
__device__ __forceinline__ void mlp_layer_vjp(const real* __restrict__ W, const real* g, real* acc_out,
                                              int ni, int no, int ln) {
  const int nip = NCH * LN;
  real acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = RL(0.0);
  const real* base = W + ln * NCH;
  int o = 0;
  for (; o + MLP_BATCH <= no; o += MLP_BATCH) {
    real w[MLP_BATCH][NCH];
#pragma unroll
    for (int u = 0; u < MLP_BATCH; ++u) load_lane_block<NCH>(base + (size_t)(o + u) * nip, w[u]);
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < MLP_BATCH; ++u) {
      const real go = g[o + u];
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] = m_fma(w[u][c], go, acc[c]);
    }
  }
  for (; o < no; ++o) {
    const real go = g[o];
    real w[NCH];
    load_lane_block<NCH>(base + (size_t)o * nip, w);
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = m_fma(w[c], go, acc[c]);
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc_out[c] = acc[c];
}

// sum over the environment's LN lanes (butterfly; every lane receives the sum)
template <int LN>
__device__ __forceinline__ real grp_sum(real x) {
#pragma unroll
  for (int off = LN / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, SIM_WAVE);
  return x;
}

// Layer normalisation of a hidden layer (App. A.2), e (LDS, n values: the ELU outputs) ->
// y (LDS): mean and population variance over the n values (each lane sums a strided share,
// then a butterfly over the environment's lanes), y = g (e - mean) / sqrt(var + eps) + beta.
// The mean and 1 / sqrt(var + eps) are left in st[0], st[1] for the input adjoint.
template <int LN>
__device__ __forceinline__ void ln_forward(const MlpArgs& P, int l, const real* e, real* y, real* st, int n, int ln) {
  real s = RL(0.0);
  for (int i = ln; i < n; i += LN) s += e[i];
  const real mu = grp_sum<LN>(s) / (real)n;
  real v = RL(0.0);
  for (int i = ln; i < n; i += LN) {
    const real d = e[i] - mu;
    v = m_fma(d, d, v);
  }
  const real var = grp_sum<LN>(v) / (real)n;
  const real is = RL(1.0) / m_sqrt(var + P.ln_eps);
  const real* g = P.lng[l];
  const real* b = P.lnb[l];
  for (int i = ln; i < n; i += LN) y[i] = m_fma(g[i], (e[i] - mu) * is, b[i]);
  if (ln == 0) {
    st[0] = mu;
    st[1] = is;
  }
  wsync();
}

// x (LDS, dims[0]) -> out (LDS, dims[nl]); hidden activations kept in h0 / h1 (<= 2 hidden).
// With layer normalisation, h0 / h1 keep the ELU outputs, the normalised layer outputs (the
// next layer's input) go through ybuf, and the mean and inverse deviation of hidden layer l
// are left in st[2 l], st[2 l + 1].
// The BF16 matrix-core layers need a whole wavefront per environment (LN = 64).
template <int LN>
__device__ __forceinline__ void mlp_forward(const MlpArgs& P, const real* x, real* h0, real* h1,
                                            real* out, uint16_t* xb, int ln, real* ybuf = nullptr,
                                            real* st = nullptr) {
  if constexpr (LN == SIM_WAVE) {
    if (P.bf16) {
      mlp_forward_bf16(P, x, h0, h1, out, xb, ln);
      return;
    }
  }
  const real* in = x;
  for (int l = 0; l < P.nl; ++l) {
    int ni = P.dims[l], no = P.dims[l + 1];
    real* dst = (l == P.nl - 1) ? out : ((l & 1) ? h1 : h0);
    bool hidden = l < P.nl - 1;
    switch (pad64(no) / LN) {
      case 1: mlp_layer_fwd<1, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 2: mlp_layer_fwd<2, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 3: mlp_layer_fwd<3, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 4: mlp_layer_fwd<4, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 5: mlp_layer_fwd<5, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 6: mlp_layer_fwd<6, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      case 7: mlp_layer_fwd<7, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
      default: mlp_layer_fwd<8, LN>(P.WT[l], P.b[l], in, dst, ni, no, hidden, ln); break;
    }
    wsync();
    in = dst;
    if (hidden && P.ln) {
      ln_forward<LN>(P, l, dst, ybuf, st + 2 * l, no, ln);
      in = ybuf;
    }
  }
}

// Given the output adjoint gout (LDS, dims[nl]) and the forward activations kept by
// mlp_forward, writes the input adjoint to xbar (LDS, dims[0]).  Scratch: gbuf (>= max width).
// The widths of a layout with LN < 64 lanes are limited to 8 * LN (the host checks).
#define SIM_MAX_NCH (SIM_MAXHID / SIM_WAVE)
template <int LN>
__device__ __forceinline__ void mlp_vjp_input(const MlpArgs& P, const real* h0, const real* h1,
                                              real* gout, real* gbuf, real* xbar, uint16_t* xb, int ln,
                                              const real* st = nullptr) {
  if constexpr (LN == SIM_WAVE) {
    if (P.bf16) {
      mlp_vjp_input_bf16(P, h0, h1, gout, gbuf, xbar, xb, ln);
      return;
    }
  }
  real* g = gout;
  for (int l = P.nl - 1; l >= 0; --l) {
    int ni = P.dims[l], no = P.dims[l + 1];
    real* dst = (l == 0) ? xbar : gbuf;
    real acc[SIM_MAX_NCH];
    switch (pad64(ni) / LN) {
      case 1: mlp_layer_vjp<1, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 2: mlp_layer_vjp<2, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 3: mlp_layer_vjp<3, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 4: mlp_layer_vjp<4, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 5: mlp_layer_vjp<5, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 6: mlp_layer_vjp<6, LN>(P.W[l], g, acc, ni, no, ln); break;
      case 7: mlp_layer_vjp<7, LN>(P.W[l], g, acc, ni, no, ln); break;
      default: mlp_layer_vjp<8, LN>(P.W[l], g, acc, ni, no, ln); break;
    }
    wsync();   // every lane has read g before dst (which may alias g) is written
    const real* hin = (l >= 1) ? (((l - 1) & 1) ? h1 : h0) : nullptr;
    const int nch = pad64(ni) / LN;
    if (hin && P.ln) {
      // through the normalisation of hidden layer l - 1: with a = (e - mean) r (r the inverse
      // deviation) and u = g * ybar, ebar = r (u - mean(u) - a mean(u a))
      const real mu = st[2 * (l - 1)], r = st[2 * (l - 1) + 1];
      const real* gg = P.lng[l - 1];
      real su = RL(0.0), sua = RL(0.0);
#pragma unroll
      for (int c = 0; c < SIM_MAX_NCH; ++c) {
        const int i = ln * nch + c;
        if (c < nch && i < ni) {
          const real u = gg[i] * acc[c];
          su += u;
          sua = m_fma(u, (hin[i] - mu) * r, sua);
        }
      }
      const real mu_u = grp_sum<LN>(su) / (real)ni, mu_ua = grp_sum<LN>(sua) / (real)ni;
#pragma unroll
      for (int c = 0; c < SIM_MAX_NCH; ++c) {
        const int i = ln * nch + c;
        if (c < nch && i < ni) {
          const real a = (hin[i] - mu) * r;
          acc[c] = r * (gg[i] * acc[c] - mu_u - a * mu_ua);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < SIM_MAX_NCH; ++c) {
      const int i = ln * nch + c;
      if (c < nch && i < ni) {
        real v = acc[c];
        if (hin) {
          real hv = hin[i];
          v *= (hv > RL(0.0)) ? RL(1.0) : (hv + RL(1.0));    // ELU'(z) = 1 (z > 0) or exp(z) = h + 1
        }
        dst[i] = v;
      }
    }
    wsync();
    g = dst;
  }
}

// --------------------------------------------------------------- policy squashing
// torques: a = tanh(y); muscle excitations: u = (tanh(y) + 1) / 2
__device__ __forceinline__ real squash(const Scal* __restrict__ m, real y) {
  real t = m_tanh(y);
  return (m->task == TASK_MTU) ? RL(0.5) * (t + RL(1.0)) : t;
}
// d(action)/dy expressed through the action value
__device__ __forceinline__ real squash_grad(const Scal* __restrict__ m, real a) {
  return (m->task == TASK_MTU) ? RL(2.0) * a * (RL(1.0) - a) : RL(1.0) - a * a;
}

// --------------------------------------------------------------- observations
// s = [q | qd | a_prev | act];  obs written to o (LDS).  The muscle task observes the
// humanoid skeleton entries (no last action), zero padding up to entry 128 and the
// muscle activations.
template <int LN>
__device__ __forceinline__ void task_obs(const Scal* __restrict__ m, const real* q, const real* qd,
                                         const real* aprev, const real* act, real* o, int ln) {
  if (m->task == TASK_NONE) {
    // no task: the observation is the state [q | qd | a_prev | act]
    const int nq = m->nq, nv = m->nv, na = m->has_last_action ? m->na : 0;
    for (int i = ln; i < nq; i += LN) o[i] = q[i];
    for (int i = ln; i < nv; i += LN) o[nq + i] = qd[i];
    for (int i = ln; i < na; i += LN) o[nq + nv + i] = aprev[i];
    for (int i = ln; i < m->n_mtu; i += LN) o[nq + nv + na + i] = act[i];
  } else if (m->task == TASK_CARTPOLE) {
    if (ln == 0) {
      real sn, cs;
      m_sincos(q[1], &sn, &cs);
      o[0] = q[0]; o[1] = qd[0]; o[2] = sn; o[3] = cs; o[4] = qd[1];
    }
  } else if (m->task == TASK_ANT || m->task == TASK_HUMANOID || m->task == TASK_MTU) {
    int nh = m->nq - 7;
    if (ln == 0) {
      real w = q[3], x = q[4], y = q[5], z = q[6];
      real n2 = w * w + x * x + y * y + z * z;
      o[0] = q[2];
      o[1] = w; o[2] = x; o[3] = y; o[4] = z;
      o[5] = qd[0]; o[6] = qd[1]; o[7] = qd[2]; o[8] = qd[3]; o[9] = qd[4]; o[10] = qd[5];
      o[11 + 2 * nh] = RL(1.0) - RL(2.0) * (x * x + y * y) / n2;       // up
      o[12 + 2 * nh] = RL(1.0) - RL(2.0) * (y * y + z * z) / n2;       // heading
    }
    for (int i = ln; i < nh; i += LN) {
      o[11 + i] = q[7 + i];
      o[11 + nh + i] = qd[6 + i];
    }
    if (m->has_last_action)
      for (int i = ln; i < m->na; i += LN) o[13 + 2 * nh + i] = aprev[i];
    if (m->task == TASK_MTU) {
      for (int i = 13 + 2 * nh + ln; i < 128; i += LN) o[i] = RL(0.0);
      for (int i = ln; i < m->n_mtu; i += LN) o[128 + i] = act[i];
    }
  }
  wsync();
}

// adjoint of task_obs: adds (d obs / d s)^T obar to (qb, qdb, abar_prev, act_bar)
template <int LN>
__device__ __forceinline__ void task_obs_vjp(const Scal* __restrict__ m, const real* q, const real* ob,
                                             real* qb, real* qdb, real* apb, real* actb, int ln) {
  if (m->task == TASK_NONE) {
    const int nq = m->nq, nv = m->nv, na = m->has_last_action ? m->na : 0;
    for (int i = ln; i < nq; i += LN) qb[i] += ob[i];
    for (int i = ln; i < nv; i += LN) qdb[i] += ob[nq + i];
    for (int i = ln; i < na; i += LN) apb[i] += ob[nq + nv + i];
    for (int i = ln; i < m->n_mtu; i += LN) actb[i] += ob[nq + nv + na + i];
  } else if (m->task == TASK_CARTPOLE) {
    if (ln == 0) {
      real sn, cs;
      m_sincos(q[1], &sn, &cs);
      qb[0] += ob[0]; qdb[0] += ob[1]; qb[1] += cs * ob[2] - sn * ob[3]; qdb[1] += ob[4];
    }
  } else if (m->task == TASK_ANT || m->task == TASK_HUMANOID || m->task == TASK_MTU) {
    int nh = m->nq - 7;
    if (ln == 0) {
      real w = q[3], x = q[4], y = q[5], z = q[6];
      real n2 = w * w + x * x + y * y + z * z;
      real i2 = RL(1.0) / n2, i4 = i2 * i2;
      real gu = ob[11 + 2 * nh], gh = ob[12 + 2 * nh];
      real u = x * x + y * y, hh = y * y + z * z;
      // up = 1 - 2u/n2 ; heading = 1 - 2hh/n2
      qb[2] += ob[0];
      qb[3] += ob[1] + gu * (RL(4.0) * u * w * i4) + gh * (RL(4.0) * hh * w * i4);
      qb[4] += ob[2] + gu * (-RL(4.0) * x * i2 + RL(4.0) * u * x * i4) + gh * (RL(4.0) * hh * x * i4);
      qb[5] += ob[3] + gu * (-RL(4.0) * y * i2 + RL(4.0) * u * y * i4) + gh * (-RL(4.0) * y * i2 + RL(4.0) * hh * y * i4);
      qb[6] += ob[4] + gu * (RL(4.0) * u * z * i4) + gh * (-RL(4.0) * z * i2 + RL(4.0) * hh * z * i4);
#pragma unroll
      for (int k = 0; k < 6; ++k) qdb[k] += ob[5 + k];
    }
    for (int i = ln; i < nh; i += LN) {
      qb[7 + i] += ob[11 + i];
      qdb[6 + i] += ob[11 + nh + i];
    }
    if (m->has_last_action)
      for (int i = ln; i < m->na; i += LN) apb[i] += ob[13 + 2 * nh + i];
    if (m->task == TASK_MTU)
      for (int i = ln; i < m->n_mtu; i += LN) actb[i] += ob[128 + i];
  }
  wsync();
}

// --------------------------------------------------------------- rewards
__device__ __forceinline__ real task_reward(const Scal* __restrict__ m, const real* q, const real* qd,
                                             const real* a, int ln) {
  real r = RL(0.0);
  if (m->task == TASK_CARTPOLE) {
    real sn, cs;
    m_sincos(q[1], &sn, &cs);
    real th = m_atan2(sn, cs);
    r = -th * th - RL(0.1) * qd[1] * qd[1] - RL(0.05) * q[0] * q[0] - RL(0.1) * qd[0] * qd[0];
  } else if (m->task == TASK_ANT || m->task == TASK_HUMANOID || m->task == TASK_MTU) {
    real w = q[3], x = q[4], y = q[5], z = q[6];
    real n2 = w * w + x * x + y * y + z * z;
    real up = RL(1.0) - RL(2.0) * (x * x + y * y) / n2;
    real hd = RL(1.0) - RL(2.0) * (y * y + z * z) / n2;
    real hgt = q[2];
    r = qd[0] + RL(0.1) * up + hd;
    if (m->task == TASK_ANT) {
      r += hgt - RL(0.27);
    } else if (m->task == TASK_HUMANOID) {
      real dh = m_fmin(m_fmax(hgt - RL(0.84), -RL(1.0)), RL(0.1));
      r += (dh < RL(0.0)) ? -RL(200.0) * dh * dh : RL(10.0) * dh;
      real aa = RL(0.0);
      for (int i = 0; i < m->na; ++i) aa += a[i] * a[i];
      r -= RL(0.002) * aa;
    } else {
      real dh = m_fmin(m_fmax(hgt - RL(0.84), -RL(1.0)), RL(0.05));
      r += (dh < RL(0.0)) ? -RL(200.0) * dh * dh : RL(4.0) * dh;
      real aa = RL(0.0);
      for (int i = 0; i < m->na; ++i) aa += a[i] * a[i];
      r -= RL(0.001) * aa;
    }
  }
  return r;
}

// adds c * dR/ds to (qb, qdb) and c * dR/da to abar
template <int LN>
__device__ __forceinline__ void task_reward_vjp(const Scal* __restrict__ m, const real* q, const real* qd,
                                                const real* a, real c, real* qb, real* qdb, real* abar,
                                                int ln) {
  if (m->task == TASK_CARTPOLE) {
    if (ln == 0) {
      real sn, cs;
      m_sincos(q[1], &sn, &cs);
      real th = m_atan2(sn, cs);
      qb[1] += c * (-RL(2.0) * th);
      qdb[1] += c * (-RL(0.2) * qd[1]);
      qb[0] += c * (-RL(0.1) * q[0]);
      qdb[0] += c * (-RL(0.2) * qd[0]);
    }
  } else if (m->task == TASK_ANT || m->task == TASK_HUMANOID || m->task == TASK_MTU) {
    if (ln == 0) {
      real w = q[3], x = q[4], y = q[5], z = q[6];
      real n2 = w * w + x * x + y * y + z * z;
      real i2 = RL(1.0) / n2, i4 = i2 * i2;
      real u = x * x + y * y, hh = y * y + z * z;
      real gu = RL(0.1) * c, gh = c;
      qb[3] += gu * (RL(4.0) * u * w * i4) + gh * (RL(4.0) * hh * w * i4);
      qb[4] += gu * (-RL(4.0) * x * i2 + RL(4.0) * u * x * i4) + gh * (RL(4.0) * hh * x * i4);
      qb[5] += gu * (-RL(4.0) * y * i2 + RL(4.0) * u * y * i4) + gh * (-RL(4.0) * y * i2 + RL(4.0) * hh * y * i4);
      qb[6] += gu * (RL(4.0) * u * z * i4) + gh * (-RL(4.0) * z * i2 + RL(4.0) * hh * z * i4);
      qdb[0] += c;
      real hgt = q[2];
      if (m->task == TASK_ANT) {
        qb[2] += c;
      } else if (m->task == TASK_HUMANOID) {
        real xh = hgt - RL(0.84);
        if (xh >= -RL(1.0) && xh <= RL(0.1)) qb[2] += c * ((xh < RL(0.0)) ? -RL(400.0) * xh : RL(10.0));
      } else {
        real xh = hgt - RL(0.84);
        if (xh >= -RL(1.0) && xh <= RL(0.05)) qb[2] += c * ((xh < RL(0.0)) ? -RL(400.0) * xh : RL(4.0));
      }
    }
    if (m->task == TASK_HUMANOID)
      for (int i = ln; i < m->na; i += LN) abar[i] += c * (-RL(0.004) * a[i]);
    if (m->task == TASK_MTU)
      for (int i = ln; i < m->na; i += LN) abar[i] += c * (-RL(0.002) * a[i]);
  }
  wsync();
}
