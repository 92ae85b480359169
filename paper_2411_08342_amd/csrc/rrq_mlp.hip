// Learned initial guess of the singularity-swap Newton solve: collection of training samples
// from the method itself, and the training kernels of the 8-64-64-2 tanh network (float32):
// forward, backward, parameter gradients, Adam.  Every reduction runs in a fixed order, so a
// training run is reproducible bit for bit.
//
// Parameter vector (the ABI layout): W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64],
// b3 [2].  The plan keeps a copy in the same layout, which the root pre-pass reads at
// wave-uniform addresses.
#include "rrq_device.h"
#include "rrq_internal.h"

namespace rrq {

// ---------------------------------------------------------------------------------------
// training samples
// ---------------------------------------------------------------------------------------

// One (pair, edge) per thread: features, chord root t_s, plain Newton from t_s.  A sample is
// kept when the chord root is inside the Bernstein ellipse of radius rho_far and Newton
// converges to a root inside it (the edges the singularity swap integrates).
// pass 0 writes flag[slot + 1] = kept; pass 1 writes the kept samples at the scanned
// positions flag[slot] (< cap).
__global__ void k_collect(PlanDev pd, TargetsDev tg, const int64_t* owner, CollectOpts co,
                          int pass, int64_t* flag, int64_t cap, float* feat, float* dt,
                          double* t0out) {
  if (input_bad(tg)) return;
  const int64_t nslot = 4 * tg.nnz;
  for (int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; slot < nslot;
       slot += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = slot >> 2;
    const int e = (int)(slot & 3);
    const int P = tg.near_patch[k];
    const int q = pd.order[P];
    const int PT = 2 * q;
    const int64_t g = owner[k];
    const double xg[3] = {tg.xyz[g], tg.xyz[tg.T + g], tg.xyz[2 * tg.T + g]};
    double xl[3];
    frame_point(pd.frame + (int64_t)P * kFrame, xg, xl);
    const double* cf = pd.edge_coef + pd.edge_off[P] + (int64_t)e * PT;   // read in place
    float f[8];
    cplx ts;
    edge_features(cf, PT, xl, f, &ts, 1, pd.E);
    const double rf = co.rho_far[q];
    int keep = 0;
    cplx t = ts;
    if (bernstein_rho(ts) <= rf) {
      int its;
      const int conv = newton_solve(cf, PT, xl, &t, co.newton_tol, co.newton_maxit, &its, 1,
                                    pd.E);
      if (t.im < 0) t.im = -t.im;
      keep = conv && bernstein_rho(t) <= rf;
    }
    if (pass == 0) {
      flag[slot + 1] = keep;
    } else if (keep) {
      const int64_t pos = flag[slot];
      if (pos < cap) {
        for (int c = 0; c < 8; ++c) feat[c * cap + pos] = f[c];
        dt[pos] = (float)(t.re - ts.re);
        dt[cap + pos] = (float)(t.im - ts.im);
        if (t0out) {
          t0out[pos] = t.re;
          t0out[cap + pos] = t.im;
        }
      }
    }
  }
}

hipError_t launch_collect(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                          const CollectOpts& co, int pass, int64_t* flag, int64_t cap,
                          float* feat, float* dt, double* t0, hipStream_t st) {
  int64_t g = (4 * tg.nnz + 255) / 256;
  if (g < 1) g = 1;
  if (pass == 0)
    hipLaunchKernelGGL(k_collect, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st, pd,
                       tg, owner, co, 0, flag, cap, feat, dt, t0);
  else
    hipLaunchKernelGGL(k_collect, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st, pd,
                       tg, owner, co, 1, flag, cap, feat, dt, t0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------------------

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", 2014)
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}


// per-block sums of x and x^2 of the 8 features and 2 targets (double)
__global__ void k_mlp_moments(const float* feat, const float* dt, int64_t m, double* part) {
  __shared__ double sm[256][20];
  double acc[20];
  for (int c = 0; c < 20; ++c) acc[c] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < 10; ++c) {
      const double v = c < 8 ? feat[c * m + i] : dt[(c - 8) * m + i];
      acc[c] += v;
      acc[10 + c] += v * v;
    }
  }
  for (int c = 0; c < 20; ++c) sm[threadIdx.x][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < 20) {
    double s = 0.0;
    for (int t = 0; t < 256; ++t) s += sm[t][threadIdx.x];
    part[blockIdx.x * 20 + threadIdx.x] = s;
  }
}

// mean and standard deviation (floor 1e-6) of the 10 columns: stats = mean[10], std[10]
__global__ void k_mlp_stats(const double* part, int nblk, int64_t m, float* stats) {
  const int c = threadIdx.x;
  if (c >= 10) return;
  double s = 0.0, s2 = 0.0;
  for (int b = 0; b < nblk; ++b) {
    s += part[b * 20 + c];
    s2 += part[b * 20 + 10 + c];
  }
  const double mean = s / (double)m;
  const double var = fmax(s2 / (double)m - mean * mean, 0.0);
  stats[c] = (float)mean;
  stats[10 + c] = (float)fmax(sqrt(var), 1e-6);
}

// Glorot-uniform weights from a counter-based generator, zero biases
__global__ void k_mlp_init(float* p, uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  int fin = 0, fout = 0;
  if (i < kMlpB1) { fin = kMlpIn; fout = kMlpH; }
  else if (i >= kMlpW2 && i < kMlpB2) { fin = kMlpH; fout = kMlpH; }
  else if (i >= kMlpW3 && i < kMlpB3) { fin = kMlpH; fout = kMlpOut; }
  if (fin == 0) { p[i] = 0.0f; return; }
  const uint64_t z = splitmix64(seed * 0x100000001B3ull + (uint64_t)i);
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  p[i] = (float)((2.0 * u - 1.0) * sqrt(6.0 / (fin + fout)));
}

// Forward pass, one sample per thread: Xn, H1, H2 [B][..], dY = 2 (Y - Yt) / B and the
// per-sample loss.  Sample b of step s is row splitmix64(seed, s, b) mod m (with
// replacement) when `sample` is set, row b otherwise; stats (may be NULL) normalise inputs
// and targets.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* p, const float* feat,
                                                 const float* dt, int64_t m, const float* stats,
                                                 int sample, uint64_t seed, int64_t step,
                                                 int B, float* Xn, float* H1, float* H2,
                                                 float* dY, float* lossb) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = p[i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int64_t row = b;
  if (sample) row = (int64_t)(splitmix64(seed * 0x2545F4914F6CDD1Dull + (uint64_t)step * (uint64_t)B + (uint64_t)b) % (uint64_t)m);
  float x[kMlpIn], h1[kMlpH];
  for (int c = 0; c < kMlpIn; ++c) {
    float v = feat[c * m + row];
    if (stats) v = (v - stats[c]) / stats[10 + c];
    x[c] = v;
    Xn[(int64_t)b * kMlpIn + c] = v;
  }
  for (int u = 0; u < kMlpH; ++u) {
    float a = w[kMlpB1 + u];
    for (int c = 0; c < kMlpIn; ++c) a += w[kMlpW1 + u * kMlpIn + c] * x[c];
    h1[u] = tanhf(a);
    H1[(int64_t)b * kMlpH + u] = h1[u];
  }
  float y[kMlpOut] = {w[kMlpB3], w[kMlpB3 + 1]};
  for (int u = 0; u < kMlpH; ++u) {
    float a = w[kMlpB2 + u];
    for (int k = 0; k < kMlpH; ++k) a += w[kMlpW2 + u * kMlpH + k] * h1[k];
    const float h2 = tanhf(a);
    H2[(int64_t)b * kMlpH + u] = h2;
    y[0] += w[kMlpW3 + u] * h2;
    y[1] += w[kMlpW3 + kMlpH + u] * h2;
  }
  float l = 0.0f;
  for (int o = 0; o < kMlpOut; ++o) {
    float t = dt[o * m + row];
    if (stats) t = (t - stats[8 + o]) / stats[18 + o];
    const float r = y[o] - t;
    dY[(int64_t)b * kMlpOut + o] = 2.0f * r / (float)B;
    l += r * r;
  }
  lossb[b] = l / (float)B;
}

// backward through the hidden layers, one sample per thread: dH2, dH1 [B][64]
__global__ __launch_bounds__(256) void k_mlp_bwd(const float* p, const float* H1,
                                                 const float* H2, const float* dY, int B,
                                                 float* dH1, float* dH2) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = p[i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float d0 = dY[(int64_t)b * kMlpOut], d1 = dY[(int64_t)b * kMlpOut + 1];
  float g2[kMlpH];
  for (int u = 0; u < kMlpH; ++u) {
    const float h = H2[(int64_t)b * kMlpH + u];
    g2[u] = (d0 * w[kMlpW3 + u] + d1 * w[kMlpW3 + kMlpH + u]) * (1.0f - h * h);
    dH2[(int64_t)b * kMlpH + u] = g2[u];
  }
  for (int k = 0; k < kMlpH; ++k) {
    float a = 0.0f;
    for (int u = 0; u < kMlpH; ++u) a += g2[u] * w[kMlpW2 + u * kMlpH + k];
    const float h = H1[(int64_t)b * kMlpH + k];
    dH1[(int64_t)b * kMlpH + k] = a * (1.0f - h * h);
  }
}

// parameter gradients, one parameter per thread, summed over the batch in order
__global__ void k_mlp_grad(const float* Xn, const float* H1, const float* H2, const float* dY,
                           const float* dH1, const float* dH2, int B, float* g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float a = 0.0f;
  if (i < kMlpB1) {
    const int u = i / kMlpIn, c = i % kMlpIn;
    for (int b = 0; b < B; ++b) a += dH1[(int64_t)b * kMlpH + u] * Xn[(int64_t)b * kMlpIn + c];
  } else if (i < kMlpW2) {
    const int u = i - kMlpB1;
    for (int b = 0; b < B; ++b) a += dH1[(int64_t)b * kMlpH + u];
  } else if (i < kMlpB2) {
    const int u = (i - kMlpW2) / kMlpH, k = (i - kMlpW2) % kMlpH;
    for (int b = 0; b < B; ++b) a += dH2[(int64_t)b * kMlpH + u] * H1[(int64_t)b * kMlpH + k];
  } else if (i < kMlpW3) {
    const int u = i - kMlpB2;
    for (int b = 0; b < B; ++b) a += dH2[(int64_t)b * kMlpH + u];
  } else if (i < kMlpB3) {
    const int o = (i - kMlpW3) / kMlpH, u = (i - kMlpW3) % kMlpH;
    for (int b = 0; b < B; ++b) a += dY[(int64_t)b * kMlpOut + o] * H2[(int64_t)b * kMlpH + u];
  } else {
    const int o = i - kMlpB3;
    for (int b = 0; b < B; ++b) a += dY[(int64_t)b * kMlpOut + o];
  }
  g[i] = a;
}

// Adam (Kingma & Ba, 2015) with bias correction; step counts from 1
__global__ void k_mlp_adam(float* p, const float* g, float* mo, float* ve, int64_t step,
                           float lr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float m = b1 * mo[i] + (1.0f - b1) * g[i];
  const float v = b2 * ve[i] + (1.0f - b2) * g[i] * g[i];
  mo[i] = m;
  ve[i] = v;
  const float mh = m / (1.0f - powf(b1, (float)step));
  const float vh = v / (1.0f - powf(b2, (float)step));
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// sum of the per-sample losses (one workgroup, fixed order)
__global__ void k_mlp_loss(const float* lossb, int B, float* out) {
  __shared__ float sm[256];
  float a = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) a += lossb[b];
  sm[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int t = 0; t < 256; ++t) s += sm[t];
    *out = s;
  }
}

// fold the input and target normalisation into the first and last layers
__global__ void k_mlp_fold(const float* p, const float* stats, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float v = p[i];
  if (i < kMlpB1) {
    v = p[i] / stats[10 + i % kMlpIn];
  } else if (i < kMlpW2) {
    const int u = i - kMlpB1;
    float a = p[i];
    for (int c = 0; c < kMlpIn; ++c) a -= p[kMlpW1 + u * kMlpIn + c] / stats[10 + c] * stats[c];
    v = a;
  } else if (i >= kMlpW3 && i < kMlpB3) {
    v = p[i] * stats[18 + (i - kMlpW3) / kMlpH];
  } else if (i >= kMlpB3) {
    const int o = i - kMlpB3;
    v = p[i] * stats[18 + o] + stats[8 + o];
  }
  out[i] = v;
}

// the plan's copy of the parameters, in the ABI layout (the root pre-pass reads it with
// wave-uniform indices)
__global__ void k_mlp_pack(const float* p, float* q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) q[i] = p[i];
}

// outputs for features [8][n] -> out [2][n] (ABI layout, one sample per thread)
__global__ __launch_bounds__(256) void k_mlp_predict(const float* p, const float* feat,
                                                     int64_t n, float* out) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = p[i];
  __syncthreads();
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * blockDim.x) {
    float x[kMlpIn], h1[kMlpH];
    for (int c = 0; c < kMlpIn; ++c) x[c] = feat[c * n + b];
    for (int u = 0; u < kMlpH; ++u) {
      float a = w[kMlpB1 + u];
      for (int c = 0; c < kMlpIn; ++c) a += w[kMlpW1 + u * kMlpIn + c] * x[c];
      h1[u] = tanhf(a);
    }
    float y0 = w[kMlpB3], y1 = w[kMlpB3 + 1];
    for (int u = 0; u < kMlpH; ++u) {
      float a = w[kMlpB2 + u];
      for (int k = 0; k < kMlpH; ++k) a += w[kMlpW2 + u * kMlpH + k] * h1[k];
      const float h2 = tanhf(a);
      y0 += w[kMlpW3 + u] * h2;
      y1 += w[kMlpW3 + kMlpH + u] * h2;
    }
    out[b] = y0;
    out[n + b] = y1;
  }
}

__global__ void k_mlp_fill0(float* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
static unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t mlp_train_run(const float* feat, const float* dt, int64_t m, int steps, int B,
                         float lr, uint64_t seed, float* params, float* loss_curve,
                         MlpScratch& s, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_moments, dim3(kMlpMomBlocks), dim3(256), 0, st, feat, dt, m, s.part);
  hipLaunchKernelGGL(k_mlp_stats, dim3(1), dim3(32), 0, st, s.part, kMlpMomBlocks, m, s.stats);
  hipLaunchKernelGGL(k_mlp_init, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, s.p, seed);
  hipLaunchKernelGGL(k_mlp_fill0, dim3(blocks_for(2 * kMlpParams, 256)), dim3(256), 0, st, s.mo,
                     2 * kMlpParams);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int it = 0; it < steps; ++it) {
    const float frac = (float)it / (float)(steps > 1 ? steps : 1);
    const float lr_s = lr * (0.05f + 0.95f * 0.5f * (1.0f + cosf(3.14159265f * frac)));
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for(B, 256)), dim3(256), 0, st, s.p, feat, dt, m,
                       s.stats, 1, seed, (int64_t)it, B, s.Xn, s.H1, s.H2, s.dY, s.lossb);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(blocks_for(B, 256)), dim3(256), 0, st, s.p, s.H1, s.H2,
                       s.dY, B, s.dH1, s.dH2);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(kMlpParams, 128)), dim3(128), 0, st, s.Xn,
                       s.H1, s.H2, s.dY, s.dH1, s.dH2, B, s.g);
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, s.p, s.g,
                       s.mo, s.mo + kMlpParams, (int64_t)it + 1, lr_s);
    if (loss_curve)
      hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, s.lossb, B, loss_curve + it);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mlp_fold, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, s.p,
                     s.stats, params);
  return hipGetLastError();
}

hipError_t mlp_loss_grad_run(const float* params, const float* feat, const float* dt,
                             int64_t n, float* loss, float* grad, MlpScratch& s,
                             hipStream_t st) {
  const int B = (int)n;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for(B, 256)), dim3(256), 0, st, params, feat, dt, n,
                     (const float*)nullptr, 0, 0ull, (int64_t)0, B, s.Xn, s.H1, s.H2, s.dY,
                     s.lossb);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(blocks_for(B, 256)), dim3(256), 0, st, params, s.H1, s.H2,
                     s.dY, B, s.dH1, s.dH2);
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(kMlpParams, 128)), dim3(128), 0, st, s.Xn,
                     s.H1, s.H2, s.dY, s.dH1, s.dH2, B, grad);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, s.lossb, B, loss);
  return hipGetLastError();
}

hipError_t mlp_predict_run(const float* params, const float* feat, int64_t n, float* out,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st,
                     params, feat, n, out);
  return hipGetLastError();
}

hipError_t mlp_pack_run(const float* params, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, params, dst);
  return hipGetLastError();
}

}  // namespace rrq
