// The learning-episode update that follows a window (Sec. 3.3, Algorithm "SHAC"): one Adam
// step of the policy, TD-lambda value estimates of the window's states from the target
// critic, the critic's mean-squared-error fit over shuffled minibatches with Adam, and the
// smooth update of the target critic.  The contractions run on the matrix cores through the
// row-contraction GEMMs of the policy-parameter gradient (sim_gemm.h).
//
// Included inside a namespace with `real` defined as float or double, after sim_math.h and
// sim_gemm.h.

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps) with bc = 1 - b^t, over every tensor of a list in
// one launch: the gradient and moments are flat with the tensors in list order, and element i
// belongs to the tensor whose range holds it
__global__ void k_adam_multi(LearnAdamT<real> A, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int t = 0;
  long base = 0;
  while (t + 1 < A.n && i >= base + A.size[t]) {
    base += A.size[t];
    ++t;
  }
  const real gi = A.g[i];
  const real m = A.b1 * A.m[i] + (RL(1.0) - A.b1) * gi;
  const real v = A.b2 * A.v[i] + (RL(1.0) - A.b2) * gi * gi;
  A.m[i] = m;
  A.v[i] = v;
  A.p[t][i - base] -= A.lr * (m / A.bc1) / (m_sqrt(v / A.bc2) + A.eps);
}

// target <- alpha target + (1 - alpha) online
__global__ void k_soft_update(real* __restrict__ t, const real* __restrict__ o, long n, real alpha) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = alpha * t[i] + (RL(1.0) - alpha) * o[i];
}

// TD-lambda estimates, one thread per env, by the backward recursion
// G_t = r_t + gamma ((1 - lambda) V_{t+1} + lambda G_{t+1}) from G_h = V_h, which equals the
// lambda-weighted average of the k-step returns of the definition.
// r [h][N], v [h+1][N] (values of s_0 .. s_h; s_0's is not used), out [h][N]
__global__ void k_td_lambda(const real* __restrict__ r, const real* __restrict__ v, const uint8_t* __restrict__ done,
                            int h, int N, real gamma, real lam, real* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  real G = v[(size_t)h * N + e];
  for (int t = h - 1; t >= 0; --t) {
    // a frame that ended in termination returns its reward alone: every k-step return from
    // it stops there and the fallen state has no value (s_{t+1} is already the reset state)
    if (done && done[(size_t)t * N + e])
      G = r[(size_t)t * N + e];
    else
      G = r[(size_t)t * N + e] + gamma * ((RL(1.0) - lam) * v[(size_t)(t + 1) * N + e] + lam * G);
    out[(size_t)t * N + e] = G;
  }
}

// minibatch rows: x[b] = obs[perm[b]], y[b] = targets[perm[b]]
// (normalised with the running statistics when given: x = (o - mean) * inv_std)
__global__ void k_gather_rows(const real* __restrict__ obs, const real* __restrict__ tgt, const int* __restrict__ perm,
                              int B, int od, const real* __restrict__ mean, const real* __restrict__ inv_std,
                              real* __restrict__ x, real* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * od) return;
  const int b = (int)(i / od), c = (int)(i % od);
  const int r = perm[b];
  real v = obs[(long)r * od + c];
  if (mean) v = (v - mean[c]) * inv_std[c];
  x[i] = v;
  if (c == 0) y[b] = tgt[r];
}

// Running observation statistics (Sec. 3.3): merges a batch of rows into the count, mean
// and (population) variance of every observation seen before, by the pairwise update of
// Chan, Golub and LeVeque: with the batch's own mean m_b and sum of squared deviations
// M2_b, delta = m_b - mean, n = count + rows,
//   mean' = mean + delta rows / n,   var' = (var count + M2_b + delta^2 count rows / n) / n,
// and inv_std = 1 / sqrt(var' + eps).  A block owns 64 columns; its 16 row groups read
// consecutive columns of a row (coalesced) and are summed in a fixed order, in FP64.  Each
// thread keeps eight independent partial sums so that eight loads are in flight at once.
#define OS_COLS 64
#define OS_GROUPS 16
#define OS_UNROLL 8

// sum over rows r = grp, grp + OS_GROUPS, ... of f(x[r][c]), in a fixed order
template <class F>
__device__ __forceinline__ double os_column_sum(const real* __restrict__ x, long rows, int od, int c, int grp, F f) {
  double p[OS_UNROLL];
#pragma unroll
  for (int u = 0; u < OS_UNROLL; ++u) p[u] = 0.0;
  long r = grp;
  for (; r + (long)(OS_UNROLL - 1) * OS_GROUPS < rows; r += (long)OS_UNROLL * OS_GROUPS) {
#pragma unroll
    for (int u = 0; u < OS_UNROLL; ++u) p[u] += f((double)x[(r + (long)u * OS_GROUPS) * od + c]);
  }
  for (; r < rows; r += OS_GROUPS) p[0] += f((double)x[r * od + c]);
  return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}
__global__ __launch_bounds__(OS_COLS * OS_GROUPS) void k_obs_stats(const real* __restrict__ x, long rows, int od,
                                                                    double count, real* __restrict__ mean,
                                                                    real* __restrict__ var, real* __restrict__ inv_std,
                                                                    double eps) {
  __shared__ double red[OS_GROUPS][OS_COLS];
  __shared__ double bmean[OS_COLS];
  const int cl = threadIdx.x % OS_COLS, grp = threadIdx.x / OS_COLS;
  const int c = blockIdx.x * OS_COLS + cl;
  const bool ok = c < od;
  double s = 0.0;
  if (ok) s = os_column_sum(x, rows, od, c, grp, [](double v) { return v; });
  red[grp][cl] = s;
  __syncthreads();
  if (grp == 0) {
    double t = 0.0;
    for (int g = 0; g < OS_GROUPS; ++g) t += red[g][cl];
    bmean[cl] = t / (double)rows;
  }
  __syncthreads();
  const double bm = bmean[cl];
  double q = 0.0;
  if (ok) q = os_column_sum(x, rows, od, c, grp, [bm](double v) { const double d = v - bm; return d * d; });
  red[grp][cl] = q;
  __syncthreads();
  if (grp == 0 && ok) {
    double m2b = 0.0;
    for (int g = 0; g < OS_GROUPS; ++g) m2b += red[g][cl];
    const double n = count + (double)rows;
    const double m0 = count > 0.0 ? (double)mean[c] : 0.0;
    const double v0 = count > 0.0 ? (double)var[c] : 0.0;
    const double delta = bm - m0;
    const double mn = m0 + delta * ((double)rows / n);
    const double vn = (v0 * count + m2b + delta * delta * (count * (double)rows / n)) / n;
    mean[c] = (real)mn;
    var[c] = (real)vn;
    inv_std[c] = (real)(1.0 / sqrt(vn + eps));
  }
}

// output adjoint of the mean squared error (1/B) sum (V - y)^2
__global__ void k_mse_seed(const real* __restrict__ V, const real* __restrict__ y, int B, real* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) d[i] = RL(2.0) / (real)B * (V[i] - y[i]);
}

// the minibatch's mean squared error before the step, by a fixed-order tree (one block)
__global__ __launch_bounds__(256) void k_mse_loss(const real* __restrict__ V, const real* __restrict__ y, int B,
                                                  real* __restrict__ out) {
  __shared__ real part[256];
  real s = RL(0.0);
  for (int i = threadIdx.x; i < B; i += 256) {
    const real d = V[i] - y[i];
    s += d * d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0] / (real)B;
}

static void launch_adam_multi(const LearnAdamT<real>& A, hipStream_t s) {
  long total = 0;
  for (int i = 0; i < A.n; ++i) total += A.size[i];
  hipLaunchKernelGGL(k_adam_multi, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, total);
}

int launch_adam(const LearnAdamT<real>& A, void* stream) {
  launch_adam_multi(A, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_soft_update(real* t, const real* o, long n, real alpha, void* stream) {
  hipLaunchKernelGGL(k_soft_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, t, o, n,
                     alpha);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_td_lambda(const real* r, const real* v, const uint8_t* done, int h, int N, real gamma, real lam,
                     real* out, void* stream) {
  hipLaunchKernelGGL(k_td_lambda, dim3((unsigned)((N + 63) / 64)), dim3(64), 0, (hipStream_t)stream, r, v, done, h,
                     N, gamma, lam, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_obs_stats(const real* x, long rows, int od, double count, real* mean, real* var, real* inv_std,
                     double eps, void* stream) {
  hipLaunchKernelGGL(k_obs_stats, dim3((unsigned)((od + OS_COLS - 1) / OS_COLS)), dim3(OS_COLS * OS_GROUPS), 0,
                     (hipStream_t)stream, x, rows, od, count, mean, var, inv_std, eps);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_critic_values(const ThetaArgsT<real>& T, real* out, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  theta_hidden(T, s);
  theta_output(T, out, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// n_iter passes over the rows in the order of perm[it], n_mb minibatches each; every
// minibatch: gather, forward, MSE seed, layer gradients, one Adam step of the critic
int launch_critic_fit(const CriticFitT<real>& F, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  ThetaArgsT<real> T = F.G;
  int step = F.adam_step;
  for (int it = 0; it < F.n_iter; ++it) {
    for (int mb = 0; mb < F.n_mb; ++mb) {
      const int r0 = (int)((long)mb * F.rows / F.n_mb), r1 = (int)((long)(mb + 1) * F.rows / F.n_mb);
      const int B = r1 - r0;
      if (B <= 0) continue;
      const long nx = (long)B * T.dims[0];
      hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, F.obs, F.targets,
                         F.perm + (long)it * F.rows + r0, B, T.dims[0], F.obs_mean, F.obs_inv_std, F.x, F.y);
      T.M = B;
      T.x0 = F.x;
      theta_hidden(T, s);
      theta_output(T, F.vbuf, s);
      if (F.loss_out)
        hipLaunchKernelGGL(k_mse_loss, dim3(1), dim3(256), 0, s, F.vbuf, F.y, B, F.loss_out + it * F.n_mb + mb);
      hipLaunchKernelGGL(k_mse_seed, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, F.vbuf, F.y, B, T.d0);
      theta_backward(T, s);
      ++step;
      const real bc1 = RL(1.0) - (real)pow((double)F.b1, (double)step);
      const real bc2 = RL(1.0) - (real)pow((double)F.b2, (double)step);
      // one Adam launch over all layers (the flat gradient holds W_0, b_0, W_1, ... in order;
      // with layer normalisation a hidden layer's gain and bias follow its W, b)
      LearnAdamT<real> A = {};
      A.n = 0;
      for (int l = 0; l < T.nl; ++l) {
        A.p[A.n] = F.W[l];
        A.size[A.n++] = (long)T.dims[l] * T.dims[l + 1];
        A.p[A.n] = F.bvec[l];
        A.size[A.n++] = T.dims[l + 1];
        if (T.ln && l + 1 < T.nl) {
          A.p[A.n] = F.lng[l];
          A.size[A.n++] = T.dims[l + 1];
          A.p[A.n] = F.lnb[l];
          A.size[A.n++] = T.dims[l + 1];
        }
      }
      A.g = T.out; A.m = F.m; A.v = F.v;
      A.lr = F.lr; A.b1 = F.b1; A.b2 = F.b2; A.eps = F.eps; A.bc1 = bc1; A.bc2 = bc2;
      launch_adam_multi(A, s);
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
