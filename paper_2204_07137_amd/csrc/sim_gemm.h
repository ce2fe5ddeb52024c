// Policy-parameter gradient of the short-horizon actor loss (App. A.1, the dL/dtheta
// term): given dL/da_t of every environment and frame, the gradient is the sum over all
// h*N (frame, env) rows of (d pi(o_t) / d theta)^T dL/da_t.  The layer inputs are the
// observations and the hidden activations that the forward window stored for every frame
// and env; the action adjoint is carried back through the squash and every ELU layer, and
// the weight gradient of a layer is the contraction of its output adjoint with its input
// over all rows.  The critic's calls (values, minibatch fit) use the same kernels and
// compute their hidden layers as GEMMs with a fused bias + ELU epilogue.
//
// Every contraction runs on the matrix cores: 32x64 output tiles staged through LDS in
// K-slices of 32, four wavefronts per tile, each wavefront a 1x2 block of 16x16x4 MFMA
// accumulators (small tiles give the 8192-row critic GEMMs two tiles per CU); the next
// slice is loaded into registers while the current one is multiplied.  Row reductions (K = h*N) are split into fixed chunks whose partial tiles
// are summed in a fixed order, so the gradient is bitwise reproducible.
//
// Included inside a namespace with `real` defined as float or double.

#define GT_M 32
#define GT_MI (GT_M / 32)   // 16-row accumulator blocks per wavefront
#define GT_N 64
#define GT_K 32
#define GT_THREADS 256

enum { EPI_STORE = 0, EPI_BIAS_ELU = 1, EPI_DELU = 2, EPI_BIAS = 3 };

typedef float mfma_v4f __attribute__((__vector_size__(4 * sizeof(float))));
typedef double mfma_v4d __attribute__((__vector_size__(4 * sizeof(double))));
typedef real mfma_v4 __attribute__((__vector_size__(4 * sizeof(real))));

__device__ __forceinline__ mfma_v4f mfma_16x16x4(float a, float b, mfma_v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma_v4d mfma_16x16x4(double a, double b, mfma_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of a 16x16 accumulator block held by lane l in element r (the column is l % 16).
// The two instructions lay their results out differently: FP32 keeps four consecutive
// rows per 16-lane group, FP64 interleaves the groups.
__device__ __forceinline__ int mfma_row(float, int l, int r) { return 4 * (l >> 4) + r; }
__device__ __forceinline__ int mfma_row(double, int l, int r) { return (l >> 4) + 4 * r; }

// C(m, n) = sum_k A(m, k) B(k, n) over k in this split's chunk, with element strides
// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn].
struct GemmArgs {
  const real* A;
  long sam, sak;
  const real* B;
  long sbk, sbn;
  int M, N, K;
  int ones_col;      // column N-1 of B is all ones (bias gradient); B holds N-1 columns
  int k_chunk;       // K rows per split (multiple of GT_K); split z = blockIdx.z
  real* C;
  long ldc, split_stride;
  int epi;
  const real* bias;  // EPI_BIAS_ELU: C = elu(acc + bias[n]); EPI_BIAS: C = acc + bias[n]
  const real* Hm;    // EPI_DELU: C = acc * elu'(z), z > 0 <=> Hm > 0, else elu'(z) = Hm + 1
  long ldh;
  // optional per-column affine on the operand loads (observation normalisation of a first
  // layer's input): A(m, k) -> (A(m, k) - a_shift[k]) * a_scale[k], B(k, n) likewise by n
  const real* a_shift;
  const real* a_scale;
  const real* b_shift;
  const real* b_scale;
};

// one K-slice of A and B into registers (zero outside the matrices and the split's chunk)
#define GT_RA (GT_M * GT_K / GT_THREADS)
#define GT_RB (GT_N * GT_K / GT_THREADS)
__device__ __forceinline__ void gemm_load_slice(const GemmArgs& g, int tid, int m0, int n0, int k0, int ke, int bcols,
                                                real (&ra)[GT_RA], real (&rb)[GT_RB]) {
  const bool a_kfast = (g.sak == 1), b_kfast = (g.sbk == 1);
#pragma unroll
  for (int r = 0; r < GT_RA; ++r) {
    const int e = tid + r * GT_THREADS;
    const int m = m0 + (a_kfast ? e / GT_K : e % GT_M), k = k0 + (a_kfast ? e % GT_K : e / GT_M);
    real v = RL(0.0);
    if (m < g.M && k < ke) {
      v = g.A[(long)m * g.sam + (long)k * g.sak];
      if (g.a_shift) v = (v - g.a_shift[k]) * g.a_scale[k];
    }
    ra[r] = v;
  }
#pragma unroll
  for (int r = 0; r < GT_RB; ++r) {
    const int e = tid + r * GT_THREADS;
    const int n = n0 + (b_kfast ? e / GT_K : e % GT_N), k = k0 + (b_kfast ? e % GT_K : e / GT_N);
    real v = RL(0.0);
    if (k < ke) {
      if (n < bcols) {
        v = g.B[(long)k * g.sbk + (long)n * g.sbn];
        if (g.b_shift) v = (v - g.b_shift[n]) * g.b_scale[n];
      } else if (g.ones_col && n == g.N - 1) v = RL(1.0);
    }
    rb[r] = v;
  }
}

__global__ __launch_bounds__(GT_THREADS) void k_gemm(GemmArgs g) {
  __shared__ real As[GT_K][GT_M + 4];
  __shared__ real Bs[GT_K][GT_N + 4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.x * GT_M, n0 = blockIdx.y * GT_N;
  const int kb = blockIdx.z * g.k_chunk;
  const int ke = min(g.K, kb + g.k_chunk);
  const int wm = (wv >> 1) * (16 * GT_MI), wn = (wv & 1) * 32;
  const int bcols = g.ones_col ? g.N - 1 : g.N;
  mfma_v4 acc[GT_MI][2];
#pragma unroll
  for (int i = 0; i < GT_MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = mfma_v4{RL(0.0), RL(0.0), RL(0.0), RL(0.0)};

  const bool a_kfast = (g.sak == 1), b_kfast = (g.sbk == 1);
  real ra[GT_RA], rb[GT_RB];
  if (kb < ke) gemm_load_slice(g, tid, m0, n0, kb, ke, bcols, ra, rb);
  for (int k0 = kb; k0 < ke; k0 += GT_K) {
#pragma unroll
    for (int r = 0; r < GT_RA; ++r) {
      const int e = tid + r * GT_THREADS;
      As[a_kfast ? e % GT_K : e / GT_M][a_kfast ? e / GT_K : e % GT_M] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < GT_RB; ++r) {
      const int e = tid + r * GT_THREADS;
      Bs[b_kfast ? e % GT_K : e / GT_N][b_kfast ? e / GT_K : e % GT_N] = rb[r];
    }
    __syncthreads();
    // the next slice's loads are in flight while this one is multiplied
    if (k0 + GT_K < ke) gemm_load_slice(g, tid, m0, n0, k0 + GT_K, ke, bcols, ra, rb);
#pragma unroll
    for (int k4 = 0; k4 < GT_K; k4 += 4) {
      const int kr = k4 + (lane >> 4);
      real b0 = Bs[kr][wn + (lane & 15)], b1 = Bs[kr][wn + 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < GT_MI; ++i) {
        const real a = As[kr][wm + 16 * i + (lane & 15)];
        acc[i][0] = mfma_16x16x4(a, b0, acc[i][0]);
        acc[i][1] = mfma_16x16x4(a, b1, acc[i][1]);
      }
    }
    __syncthreads();
  }
  real* C = g.C + (long)blockIdx.z * g.split_stride;
#pragma unroll
  for (int i = 0; i < GT_MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + mfma_row(RL(0.0), lane, r);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          real v = acc[i][j][r];
          if (g.epi == EPI_BIAS_ELU) {
            v += g.bias[n];
            v = v > RL(0.0) ? v : m_expm1(v);
          } else if (g.epi == EPI_BIAS) {
            v += g.bias[n];
          } else if (g.epi == EPI_DELU) {
            const real hv = g.Hm[(long)m * g.ldh + n];
            v *= hv > RL(0.0) ? RL(1.0) : hv + RL(1.0);
          }
          C[(long)m * g.ldc + n] = v;
        }
      }
}

// adjoint of the pre-squash policy output: dL/dy = dL/da da/dy with a = tanh(y) (1 - a^2)
// or, for muscle excitations, u = (tanh(y) + 1) / 2 (2 u (1 - u))
__global__ void k_theta_seed(const real* __restrict__ da, const real* __restrict__ a, real* __restrict__ d, long n,
                             int mtu) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const real av = a[i];
    d[i] = da[i] * (mtu ? RL(2.0) * av * (RL(1.0) - av) : RL(1.0) - av * av);
  }
}

// dL/dlog_std[i] = sum over rows of dL/dy[row][i] exp(log_std[i]) eps[row][i] (the
// reparameterised sample y = mu + exp(log_std) eps); one block per action, a fixed-order
// tree over 256 per-thread partial sums, so the result is reproducible
__global__ __launch_bounds__(256) void k_log_std_grad(const real* __restrict__ d, const real* __restrict__ eps,
                                                      const real* __restrict__ log_std, long rows, int na,
                                                      real* __restrict__ out) {
  __shared__ real part[256];
  const int i = blockIdx.x, tid = threadIdx.x;
  real s = RL(0.0);
  for (long r = tid; r < rows; r += 256) s += d[r * na + i] * eps[r * na + i];
  part[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[i] = part[0] * m_exp(log_std[i]);
}

// sum of the split partials in split order; column `in` of each row is the bias gradient
__global__ void k_split_reduce(const real* __restrict__ part, int splits, long stride, int rows, int cols,
                               real* __restrict__ gW, real* __restrict__ gb) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  real s = RL(0.0);
  for (int z = 0; z < splits; ++z) s += part[z * stride + idx];
  const int o = (int)(idx / cols), i = (int)(idx % cols);
  if (i < cols - 1) gW[(long)o * (cols - 1) + i] = s;
  else gb[o] = s;
}

// ---- layer normalisation of the hidden layers (App. A.2) in the policy-gradient pass
// the normalised layer inputs from the window's ELU outputs and per-row statistics (the window's
// own expression, so the values are those its actor consumed)
__global__ void k_ln_apply(const real* __restrict__ E, long lde, const real* __restrict__ st, long ldst, int j,
                           const real* __restrict__ g, const real* __restrict__ b, real* __restrict__ Y, long M,
                           int n) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * n) return;
  const long r = idx / n;
  const int c = (int)(idx % n);
  const real mu = st[r * ldst + 2 * j], is = st[r * ldst + 2 * j + 1];
  Y[idx] = m_fma(g[c], (E[r * lde + c] - mu) * is, b[c]);
}

// Layer normalisation of hidden layer j row by row, computing its statistics (the critic's
// passes, which have no window activations): one wavefront per row; lane c sums columns c,
// c + 64, ... and a butterfly over the wavefront gives the row's mean and population
// variance; st[r ldst + 2 j] / [.. + 1] receive the mean and 1 / sqrt(var + eps), and
// Y [M][n] = g (E - mean) / sqrt(var + eps) + b as k_ln_apply forms it.
__global__ __launch_bounds__(256) void k_ln_forward(const real* __restrict__ E, long lde, real* __restrict__ st,
                                                    long ldst, int j, const real* __restrict__ g,
                                                    const real* __restrict__ b, real* __restrict__ Y, long M, int n,
                                                    real eps) {
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const long r = (long)blockIdx.x * 4 + wave;
  if (r >= M) return;   // uniform over the wavefront
  const real* e = E + r * lde;
  real sm = RL(0.0);
  for (int c = lane; c < n; c += SIM_WAVE) sm += e[c];
#pragma unroll
  for (int o = SIM_WAVE / 2; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  const real mu = sm / (real)n;
  real sv2 = RL(0.0);
  for (int c = lane; c < n; c += SIM_WAVE) {
    const real d = e[c] - mu;
    sv2 = m_fma(d, d, sv2);
  }
#pragma unroll
  for (int o = SIM_WAVE / 2; o > 0; o >>= 1) sv2 += __shfl_xor(sv2, o);
  const real is = RL(1.0) / m_sqrt(sv2 / (real)n + eps);
  for (int c = lane; c < n; c += SIM_WAVE) Y[r * n + c] = m_fma(g[c], (e[c] - mu) * is, b[c]);
  if (lane == 0) {
    st[r * ldst + 2 * j] = mu;
    st[r * ldst + 2 * j + 1] = is;
  }
}

// Adjoint through the normalisation and the ELU of hidden layer j, row by row: dY [M][n] (the
// adjoint of the normalised outputs) -> D [M][n] (the adjoint of the pre-activations), with
// a = (e - mean) r and u = g dY, ebar = r (u - mean(u) - a mean(u a)), D = ebar ELU'(z).  One
// wavefront per row at a time (lane c holds columns c, c + 64, ...); each block also sums, over
// its rows in a fixed order, dY a (the gain gradient) and dY (the bias gradient) per column
// into part[block][0 / 1][n], reduced across blocks in block order by k_ln_reduce.
#define SIM_LN_Q (SIM_MAXHID / SIM_WAVE)
__global__ __launch_bounds__(256) void k_ln_backward(const real* __restrict__ dY, const real* __restrict__ E, long lde,
                                                     const real* __restrict__ st, long ldst, int j,
                                                     const real* __restrict__ g, real* __restrict__ D, long M, int n,
                                                     real* __restrict__ part) {
  __shared__ real red[4][2][SIM_MAXHID];
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  real pg[SIM_LN_Q], pb[SIM_LN_Q];
#pragma unroll
  for (int q = 0; q < SIM_LN_Q; ++q) { pg[q] = RL(0.0); pb[q] = RL(0.0); }
  for (long r = (long)blockIdx.x * 4 + wave; r < M; r += (long)gridDim.x * 4) {
    const real mu = st[r * ldst + 2 * j], is = st[r * ldst + 2 * j + 1];
    real u[SIM_LN_Q], a[SIM_LN_Q], ev[SIM_LN_Q];
    real su = RL(0.0), sua = RL(0.0);
#pragma unroll
    for (int q = 0; q < SIM_LN_Q; ++q) {
      const int c = lane + SIM_WAVE * q;
      u[q] = a[q] = ev[q] = RL(0.0);
      if (c < n) {
        const real dy = dY[r * n + c];
        ev[q] = E[r * lde + c];
        a[q] = (ev[q] - mu) * is;
        u[q] = g[c] * dy;
        su += u[q];
        sua = m_fma(u[q], a[q], sua);
        pg[q] = m_fma(dy, a[q], pg[q]);
        pb[q] += dy;
      }
    }
    const real mu_u = wave_sum(su) / (real)n, mu_ua = wave_sum(sua) / (real)n;
#pragma unroll
    for (int q = 0; q < SIM_LN_Q; ++q) {
      const int c = lane + SIM_WAVE * q;
      if (c < n) {
        const real eb = is * (u[q] - mu_u - a[q] * mu_ua);
        D[r * n + c] = eb * ((ev[q] > RL(0.0)) ? RL(1.0) : ev[q] + RL(1.0));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < SIM_LN_Q; ++q) {
    const int c = lane + SIM_WAVE * q;
    if (c < n) { red[wave][0][c] = pg[q]; red[wave][1][c] = pb[q]; }
  }
  __syncthreads();
  for (int c = (int)threadIdx.x; c < n; c += 256) {
    part[((long)blockIdx.x * 2 + 0) * n + c] = ((red[0][0][c] + red[1][0][c]) + red[2][0][c]) + red[3][0][c];
    part[((long)blockIdx.x * 2 + 1) * n + c] = ((red[0][1][c] + red[1][1][c]) + red[2][1][c]) + red[3][1][c];
  }
}

__global__ void k_ln_reduce(const real* __restrict__ part, int nb, int n, real* __restrict__ gg,
                            real* __restrict__ gb) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= n) return;
  real s0 = RL(0.0), s1 = RL(0.0);
  for (int z = 0; z < nb; ++z) {
    s0 += part[((long)z * 2 + 0) * n + c];
    s1 += part[((long)z * 2 + 1) * n + c];
  }
  gg[c] = s0;
  gb[c] = s1;
}

static void launch_gemm(const GemmArgs& g, int splits, hipStream_t s) {
  dim3 grid((g.M + GT_M - 1) / GT_M, (g.N + GT_N - 1) / GT_N, splits);
  hipLaunchKernelGGL(k_gemm, grid, dim3(GT_THREADS), 0, s, g);
}

// the hidden layers of the network on T.M rows of T.x0 (H[l + 1] = elu(H[l] W_l^T + b_l))
static void theta_hidden(const ThetaArgsT<real>& T, hipStream_t s) {
  const int M = T.M, L = T.nl;
  for (int l = 0; l + 1 < L; ++l) {
    const int ni = T.dims[l], no = T.dims[l + 1];
    GemmArgs g = {};
    g.A = (l == 0) ? T.x0 : (T.ln ? T.Y[l] : T.H[l]);
    g.sam = ni; g.sak = 1;
    g.B = T.W[l]; g.sbk = 1; g.sbn = ni;
    g.M = M; g.N = no; g.K = ni;
    g.k_chunk = (ni + GT_K - 1) / GT_K * GT_K;
    g.C = T.H[l + 1]; g.ldc = no;
    g.epi = EPI_BIAS_ELU; g.bias = T.b[l];
    if (l == 0) { g.a_shift = T.x_shift; g.a_scale = T.x_scale; }
    launch_gemm(g, 1, s);
    if (T.ln)
      hipLaunchKernelGGL(k_ln_forward, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, T.H[l + 1], (long)no, T.st,
                         T.ldst, l, T.lng[l], T.lnb[l], T.Y[l + 1], (long)M, no, T.ln_eps);
  }
}

// the linear output layer on the rows (out [M][dims[L]] = H[L-1] W^T + b)
static void theta_output(const ThetaArgsT<real>& T, real* out, hipStream_t s) {
  const int L = T.nl, ni = T.dims[L - 1], no = T.dims[L];
  GemmArgs g = {};
  g.A = (L == 1) ? T.x0 : (T.ln ? T.Y[L - 1] : T.H[L - 1]);
  g.sam = ni; g.sak = 1;
  g.B = T.W[L - 1]; g.sbk = 1; g.sbn = ni;
  g.M = T.M; g.N = no; g.K = ni;
  g.k_chunk = (ni + GT_K - 1) / GT_K * GT_K;
  g.C = out; g.ldc = no;
  g.epi = EPI_BIAS; g.bias = T.b[L - 1];
  if (L == 1) { g.a_shift = T.x_shift; g.a_scale = T.x_scale; }
  launch_gemm(g, 1, s);
}

// given the output adjoint in T.d0, every layer's weight and bias gradient (flat in T.out)
static void theta_backward(const ThetaArgsT<real>& T, hipStream_t s) {
  const int M = T.M, L = T.nl;
  real* dcur = T.d0;
  real* dnext = T.d1;
  const int chunk = ((M + T.splits - 1) / T.splits + GT_K - 1) / GT_K * GT_K;
  const int splits = (M + chunk - 1) / chunk;
  for (int l = L - 1; l >= 0; --l) {
    const int ni = T.dims[l], no = T.dims[l + 1];
    // layer l's input: the observations, the hidden activations, or their normalisations
    const real* xin = (l == 0) ? T.x0 : (T.ln ? T.Y[l] : T.H[l]);
    const long ldx = (l > 0 && !T.ln && T.ldH[l]) ? T.ldH[l] : ni;
    const long ldh = (l > 0 && T.ldH[l]) ? T.ldH[l] : ni;
    GemmArgs g = {};
    g.A = dcur; g.sam = 1; g.sak = no;
    g.B = xin; g.sbk = ldx; g.sbn = 1; g.ones_col = 1;
    g.M = no; g.N = ni + 1; g.K = M; g.k_chunk = chunk;
    g.C = T.part; g.ldc = ni + 1; g.split_stride = (long)no * (ni + 1);
    g.epi = EPI_STORE;
    if (l == 0) { g.b_shift = T.x_shift; g.b_scale = T.x_scale; }
    launch_gemm(g, splits, s);
    const long nr = (long)no * (ni + 1);
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, T.part, splits,
                       (long)no * (ni + 1), no, ni + 1, T.out + T.off_w[l], T.out + T.off_b[l]);
    if (l > 0) {
      GemmArgs g2 = {};
      g2.A = dcur; g2.sam = no; g2.sak = 1;
      g2.B = T.W[l]; g2.sbk = ni; g2.sbn = 1;
      g2.M = M; g2.N = ni; g2.K = no;
      g2.k_chunk = (no + GT_K - 1) / GT_K * GT_K;
      g2.C = dnext; g2.ldc = ni;
      if (!T.ln) {
        g2.epi = EPI_DELU; g2.Hm = T.H[l]; g2.ldh = ldh;
        launch_gemm(g2, 1, s);
        real* t = dcur; dcur = dnext; dnext = t;
      } else {
        // the adjoint of the normalised outputs, then through the normalisation and the ELU
        // into dcur (whose layer-l adjoint has been consumed)
        g2.epi = EPI_STORE;
        launch_gemm(g2, 1, s);
        hipLaunchKernelGGL(k_ln_backward, dim3(T.ln_blocks), dim3(256), 0, s, dnext, T.H[l], ldh, T.st, T.ldst, l - 1,
                           T.lng[l - 1], dcur, (long)M, ni, T.lnpart);
        hipLaunchKernelGGL(k_ln_reduce, dim3((ni + 255) / 256), dim3(256), 0, s, T.lnpart, T.ln_blocks, ni,
                           T.out + T.off_g[l - 1], T.out + T.off_beta[l - 1]);
      }
    }
  }
}

int launch_theta(const ThetaArgsT<real>& T, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int M = T.M, L = T.nl;
  // the hidden layers on the stored observations, unless the window stored them
  if (!T.hidden_given) {
    if (T.ln) return -1;   // normalised layers: only the window's own activations
    theta_hidden(T, s);
  }
  if (T.ln)
    for (int l = 1; l < L; ++l) {
      const long n = (long)M * T.dims[l];
      hipLaunchKernelGGL(k_ln_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T.H[l], T.ldH[l], T.st,
                         T.ldst, l - 1, T.lng[l - 1], T.lnb[l - 1], T.Y[l], (long)M, T.dims[l]);
    }
  const int na = T.dims[L];
  const long nseed = (long)M * na;
  hipLaunchKernelGGL(k_theta_seed, dim3((unsigned)((nseed + 255) / 256)), dim3(256), 0, s, T.da, T.act, T.d0, nseed,
                     T.mtu);
  if (T.noise && T.out_log_std)
    hipLaunchKernelGGL(k_log_std_grad, dim3(na), dim3(256), 0, s, T.d0, T.noise, T.log_std, (long)M, na,
                       T.out_log_std);
  theta_backward(T, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
