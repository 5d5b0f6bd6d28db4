// selector.hip -- per-graph choice between GConn+Euler and BFS by a small MLP.
//
// Features of graph g (8 values):  log n, log(1+m), mean degree,
// log(1+variance of degree), log(1+max degree), and for three seeded sources
// log2(1 + depth reached by a capped BFS): the BFS stops at kProbeLevels
// levels, at the source's eccentricity, or at the first level whose ball
// (vertices within that many hops) holds kProbeBall vertices, so a probe
// costs at most about kProbeBall vertices' arcs whatever the graph (an
// uncapped search visits all of a low-diameter graph: three of them over a
// 4096-graph batch took longer than its spanning forests).  The degree
// moments are one segmented reduction (a block per graph); each probe is one
// workgroup that keeps the visited set and the frontier in LDS.
//
// Network: 8 -> 64 -> 64 -> 2, ReLU, fp32, inputs z-scored with stored
// statistics; logit 0 = GConn+Euler, logit 1 = BFS; the larger logit wins and
// ties or non-finite features fall back to GConn+Euler.  Parameters are one
// float array in the order W1[64][8], b1[64], W2[64][64], b2[64], W3[2][64],
// b3[2] (4866 floats).  Training runs on the device too: one block per sample
// computes the forward pass, the weighted softmax cross-entropy and its
// gradient with respect to every parameter; a second kernel averages the
// per-sample gradients in a fixed order (deterministic), and a third applies
// Adam (Kingma & Ba, 2015).
#include "rst_internal.h"
#include "device_common.h"

#include <cmath>
#include <cstring>
#include <new>

namespace rst {

constexpr int kIn = 8, kH = 64, kOut = 2;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kOut * kH,
              kParams = kOffB3 + kOut;
static_assert(kParams == 4866, "parameter layout");
constexpr int kProbeLevels = 64;
constexpr int kProbes = 3;
constexpr int kProbeBall = 1024;     // a probe stops once its ball holds this many vertices
constexpr int kProbeThreads = 256;
constexpr int kProbeHash = 4096;     // visited set: < kProbeBall + kProbeThreads keys
static_assert(kProbeHash >= 2 * (kProbeBall + kProbeThreads), "probe hash load");

struct Selector {
  float *dev = nullptr;   // [16 + kParams]: mean[8], std[8], parameters
};

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_degree_moments(const OffT *__restrict__ off,
                                                           const int64_t *__restrict__ vtx_off,
                                                           float *feat) {
  __shared__ double s_sum[kBlock], s_sq[kBlock];
  __shared__ int64_t s_max[kBlock];
  const int g = blockIdx.x;
  const int64_t b = vtx_off[g], e = vtx_off[g + 1];
  double sum = 0.0, sq = 0.0;
  int64_t mx = 0;
  for (int64_t v = b + threadIdx.x; v < e; v += kBlock) {
    const int64_t d = (int64_t)(off[v + 1] - off[v]);
    sum += (double)d;
    sq += (double)d * (double)d;
    mx = d > mx ? d : mx;
  }
  s_sum[threadIdx.x] = sum; s_sq[threadIdx.x] = sq; s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {     // fixed-order tree: deterministic
    if ((int)threadIdx.x < o) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
      s_sq[threadIdx.x] += s_sq[threadIdx.x + o];
      s_max[threadIdx.x] = s_max[threadIdx.x] > s_max[threadIdx.x + o] ? s_max[threadIdx.x]
                                                                       : s_max[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nv = (double)(e - b);
    const double mean = nv > 0 ? s_sum[0] / nv : 0.0;
    double var = nv > 0 ? s_sq[0] / nv - mean * mean : 0.0;
    var = var < 0 ? 0 : var;
    float *f = feat + (int64_t)g * kIn;
    f[0] = (float)log(nv > 1 ? nv : 1.0);
    f[1] = (float)log(1.0 + s_sum[0] / 2.0);
    f[2] = (float)mean;
    f[3] = (float)log1p(var);
    f[4] = (float)log1p((double)s_max[0]);
  }
}

// splitmix64 (Steele, Lea, Flood, OOPSLA 2014): the state is advanced by the
// golden-ratio increment and finalised.  splitmix64((k - 1) * gamma) is the
// k-th output of the generator seeded with 0.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// One probe per workgroup: graph g = blockIdx.x / kProbes, probe s =
// blockIdx.x % kProbes, source vtx_off[g] + (the (3g + s + 1)-th output of
// splitmix64 seeded with 0) mod n_g.  Level after level the frontier's arcs
// are walked with unit stride (degree prefix in LDS); a neighbour not yet in
// the LDS hash set of visited vertices joins the next frontier.  The probe
// stops at kProbeLevels levels, when the next frontier is empty, or once the
// visited vertices number kProbeBall (the level that reached it counts).
template <class OffT>
__global__ __launch_bounds__(kProbeThreads) void k_probe(const OffT *__restrict__ off,
                                                         const int32_t *__restrict__ cols,
                                                         const int64_t *__restrict__ vtx_off,
                                                         float *feat) {
  __shared__ int32_t keys[kProbeHash];
  __shared__ int32_t fr[2][kProbeBall];
  __shared__ OffT beg[kProbeBall];
  __shared__ int32_t sc[kProbeBall + 1];
  __shared__ int s_wave[kProbeThreads / kWave];
  __shared__ int s_new;
  const int t = threadIdx.x;
  const int g = blockIdx.x / kProbes, s = blockIdx.x % kProbes;
  const int64_t b = vtx_off[g], n = vtx_off[g + 1] - b;
  for (int i = t; i < kProbeHash; i += kProbeThreads) keys[i] = -1;
  int depth = 0;
  if (n > 0) {
    const uint64_t h = splitmix64(((uint64_t)g * kProbes + (uint64_t)s) * 0x9E3779B97F4A7C15ull);
    const int32_t src = (int32_t)(b + (int64_t)(h % (uint64_t)n));
    __syncthreads();
    auto insert = [&](int32_t w) -> bool {   // true if w was not in the set
      uint32_t hh = ((uint32_t)w * 0x9E3779B1u) >> (32 - 12);
      while (true) {
        const int32_t old = atomicCAS(&keys[hh], -1, w);
        if (old == -1) return true;
        if (old == w) return false;
        hh = (hh + 1) & (kProbeHash - 1);
      }
    };
    if (t == 0) { insert(src); fr[0][0] = src; }
    int c = 0, nf = 1, total = 1;
    while (depth < kProbeLevels) {
      // degree prefix of the frontier (at most kProbeBall vertices, 4 per thread)
      int d[kProbeBall / kProbeThreads];
      int mine = 0;
#pragma unroll
      for (int q = 0; q < kProbeBall / kProbeThreads; ++q) {
        const int i = t * (kProbeBall / kProbeThreads) + q;
        d[q] = 0;
        if (i < nf) {
          const int32_t u = fr[c][i];
          const OffT bu = off[u];
          d[q] = (int)(off[u + 1] - bu);
          beg[i] = bu;
        }
        mine += d[q];
      }
      int arcs;
      int run = block_excl_scan<kProbeThreads>(mine, s_wave, &arcs);
#pragma unroll
      for (int q = 0; q < kProbeBall / kProbeThreads; ++q) {
        const int i = t * (kProbeBall / kProbeThreads) + q;
        if (i < nf) sc[i] = run;
        run += d[q];
      }
      if (t == 0) { sc[nf] = arcs; s_new = 0; }
      __syncthreads();
      for (int k0 = 0; k0 < arcs; k0 += kProbeThreads) {
        const int k = k0 + t;
        if (k < arcs) {
          const int j = lds_upper_search(sc, nf, k);
          const int32_t w = cols[beg[j] + (OffT)(k - sc[j])];
          if (insert(w)) {
            const int idx = atomicAdd(&s_new, 1);
            if (idx < kProbeBall) fr[c ^ 1][idx] = w;
          }
        }
        __syncthreads();
        if (total + s_new >= kProbeBall) break;   // the ball is full: this level ends the probe
      }
      const int nn = s_new;
      __syncthreads();                            // s_new, sc and beg are rewritten next level
      if (nn == 0) break;                         // the source's eccentricity
      ++depth;
      total += nn;
      if (total >= kProbeBall) break;
      c ^= 1;
      nf = nn;
    }
  }
  if (t == 0) feat[(int64_t)g * kIn + 5 + s] = log2f(1.0f + (float)depth);
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------

// One block of kH threads per sample: activations in LDS.
__device__ __forceinline__ void mlp_forward_block(const float *__restrict__ P, const float *x,
                                                  float *h1, float *h2, float *z) {
  const int j = threadIdx.x;
  float a = P[kOffB1 + j];
#pragma unroll
  for (int k = 0; k < kIn; ++k) a += P[kOffW1 + j * kIn + k] * x[k];
  h1[j] = a > 0.f ? a : 0.f;
  __syncthreads();
  a = P[kOffB2 + j];
  for (int k = 0; k < kH; ++k) a += P[kOffW2 + j * kH + k] * h1[k];
  h2[j] = a > 0.f ? a : 0.f;
  __syncthreads();
  if (j < kOut) {
    float o = P[kOffB3 + j];
    for (int k = 0; k < kH; ++k) o += P[kOffW3 + j * kH + k] * h2[k];
    z[j] = o;
  }
  __syncthreads();
}

__device__ __forceinline__ void load_normalised(const float *__restrict__ norm,
                                                const float *__restrict__ X, int64_t b, float *x) {
  if ((int)threadIdx.x < kIn) {
    const float sd = norm[kIn + threadIdx.x];
    x[threadIdx.x] = (X[b * kIn + threadIdx.x] - norm[threadIdx.x]) / (sd > 1e-6f ? sd : 1e-6f);
  }
  __syncthreads();
}

__global__ __launch_bounds__(kH) void k_mlp_forward(int64_t B, const float *__restrict__ norm,
                                                    const float *__restrict__ P,
                                                    const float *__restrict__ X, float *logits,
                                                    uint8_t *choice) {
  __shared__ float x[kIn], h1[kH], h2[kH], z[kOut];
  const int64_t b = blockIdx.x;
  load_normalised(norm, X, b, x);
  mlp_forward_block(P, x, h1, h2, z);
  if (threadIdx.x == 0) {
    if (logits) { logits[b * kOut] = z[0]; logits[b * kOut + 1] = z[1]; }
    if (choice) {
      bool finite = true;
      for (int k = 0; k < kIn; ++k) finite = finite && isfinite(X[b * kIn + k]);
      choice[b] = (finite && isfinite(z[0]) && isfinite(z[1]) && z[1] > z[0]) ? 1 : 0;
    }
  }
}

// Weighted softmax cross-entropy of one sample and its gradient with respect to
// every parameter, written to G[b][kParams]; loss[b] = w * (-log p_y).
__global__ __launch_bounds__(kH) void k_mlp_grad(int64_t B, const float *__restrict__ norm,
                                                 const float *__restrict__ P,
                                                 const float *__restrict__ X,
                                                 const int32_t *__restrict__ y,
                                                 const float *__restrict__ wt, float *Gr,
                                                 float *loss) {
  __shared__ float x[kIn], h1[kH], h2[kH], z[kOut], dz[kOut], dh2[kH];
  const int64_t b = blockIdx.x;
  const int j = threadIdx.x;
  load_normalised(norm, X, b, x);
  mlp_forward_block(P, x, h1, h2, z);
  const float w = wt[b];
  const int yb = y[b];
  if (j == 0) {
    const float mz = z[0] > z[1] ? z[0] : z[1];
    const float e0 = expf(z[0] - mz), e1 = expf(z[1] - mz);
    const float s = e0 + e1;
    const float p0 = e0 / s, p1 = e1 / s;
    loss[b] = -w * (logf(yb == 0 ? p0 : p1));
    dz[0] = w * (p0 - (yb == 0 ? 1.f : 0.f));
    dz[1] = w * (p1 - (yb == 1 ? 1.f : 0.f));
  }
  __syncthreads();
  float *g = Gr + b * kParams;
  // output layer
  for (int o = 0; o < kOut; ++o) g[kOffW3 + o * kH + j] = dz[o] * h2[j];
  if (j < kOut) g[kOffB3 + j] = dz[j];
  float d2 = 0.f;
  for (int o = 0; o < kOut; ++o) d2 += P[kOffW3 + o * kH + j] * dz[o];
  d2 = h2[j] > 0.f ? d2 : 0.f;
  dh2[j] = d2;
  __syncthreads();
  // second layer: row j of W2
  for (int k = 0; k < kH; ++k) g[kOffW2 + j * kH + k] = dh2[j] * h1[k];
  g[kOffB2 + j] = dh2[j];
  float d1 = 0.f;
  for (int k = 0; k < kH; ++k) d1 += P[kOffW2 + k * kH + j] * dh2[k];
  d1 = h1[j] > 0.f ? d1 : 0.f;
  for (int k = 0; k < kIn; ++k) g[kOffW1 + j * kIn + k] = d1 * x[k];
  g[kOffB1 + j] = d1;
}

// grad[p] = (1/B) sum_b G[b][p], summed in index order; loss_mean likewise.
__global__ __launch_bounds__(kBlock) void k_grad_mean(int64_t B, const float *__restrict__ Gr,
                                                      const float *__restrict__ loss, float *grad,
                                                      float *loss_mean) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) {
    float acc = 0.f;
    for (int64_t b = 0; b < B; ++b) acc += Gr[b * kParams + p];
    grad[p] = acc / (float)B;
  }
  if (p == kParams && loss_mean) {
    float acc = 0.f;
    for (int64_t b = 0; b < B; ++b) acc += loss[b];
    *loss_mean = acc / (float)B;
  }
}

__global__ __launch_bounds__(kBlock) void k_adam(float *P, const float *__restrict__ grad, float *m,
                                                 float *v, float lr, float beta1, float beta2,
                                                 float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = grad[p];
  const float mp = beta1 * m[p] + (1.f - beta1) * g;
  const float vp = beta2 * v[p] + (1.f - beta2) * g * g;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
}

// column mean / standard deviation of X[B][8] into norm[16] (fp64 accumulation)
__global__ void k_feature_stats(int64_t B, const float *__restrict__ X, float *norm) {
  const int k = threadIdx.x;
  if (k >= kIn) return;
  double s = 0.0, q = 0.0;
  for (int64_t b = 0; b < B; ++b) { const double x = X[b * kIn + k]; s += x; q += x * x; }
  const double mean = B > 0 ? s / (double)B : 0.0;
  double var = B > 0 ? q / (double)B - mean * mean : 0.0;
  norm[k] = (float)mean;
  norm[kIn + k] = (float)sqrt(var > 0 ? var : 0.0);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

rst_status enqueue_features(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, float *feat) {
  const int32_t G = b->num_graphs;
  const unsigned probes = (unsigned)G * kProbes;
  if (g->offset_bytes == 4) {
    hipLaunchKernelGGL(k_degree_moments<int32_t>, dim3((unsigned)G), dim3(kBlock), 0, ctx->stream,
                       (const int32_t *)g->offsets, b->vtx_off, feat);
    hipLaunchKernelGGL(k_probe<int32_t>, dim3(probes), dim3(kProbeThreads), 0, ctx->stream,
                       (const int32_t *)g->offsets, g->cols, b->vtx_off, feat);
  } else {
    hipLaunchKernelGGL(k_degree_moments<int64_t>, dim3((unsigned)G), dim3(kBlock), 0, ctx->stream,
                       (const int64_t *)g->offsets, b->vtx_off, feat);
    hipLaunchKernelGGL(k_probe<int64_t>, dim3(probes), dim3(kProbeThreads), 0, ctx->stream,
                       (const int64_t *)g->offsets, g->cols, b->vtx_off, feat);
  }
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_mlp_forward(rst_ctx *ctx, int64_t B, const float *norm, const float *params,
                               const float *X, float *logits, uint8_t *choice) {
  if (B <= 0) return RST_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)B), dim3(kH), 0, ctx->stream, B, norm, params, X,
                     logits, choice);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status run_selector(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, uint8_t *choice) {
  const int32_t G = b->num_graphs;
  float *feat = ws_take<float>(ctx, (size_t)G * kIn);
  RST_TRY(enqueue_features(ctx, g, b, feat));
  return enqueue_mlp_forward(ctx, G, ctx->selector->dev, ctx->selector->dev + 16, feat, nullptr,
                             choice);
}

size_t selector_scratch_bytes(const rst_ctx *ctx, const rst_csr *g, int32_t G) {
  (void)ctx;
  (void)g;
  return ws_bytes((size_t)G * kIn, 4);
}

const void *selector_weights(const rst_ctx *ctx) {
  return ctx->selector ? ctx->selector->dev : nullptr;
}

void selector_free(rst_ctx *ctx) {
  if (ctx->selector) {
    if (ctx->selector->dev) (void)hipFree(ctx->selector->dev);
    delete ctx->selector;
    ctx->selector = nullptr;
  }
}

}  // namespace rst

using namespace rst;

extern "C" {

rst_status rst_features(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, float *feat) {
  if (!ctx || !b || !feat || b->num_graphs < 1 || !b->vtx_off) return RST_E_INVAL;
  if (!g || g->n < 1 || !g->offsets || (g->offset_bytes != 4 && g->offset_bytes != 8))
    return RST_E_INVAL;
  if (g->nnz > 0 && !g->cols) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  RST_TRY(enqueue_features(ctx, g, b, feat));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

rst_status rst_feature_stats(rst_ctx *ctx, const float *X, int64_t B, float *norm) {
  if (!ctx || !X || !norm || B < 1) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(kIn), 0, ctx->stream, B, X, norm);
  RST_HIP(hipGetLastError());
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

rst_status rst_mlp_forward(rst_ctx *ctx, const float *norm, const float *params, const float *X,
                           int64_t B, float *logits, uint8_t *choice) {
  if (!ctx || !norm || !params || !X || B < 0 || (!logits && !choice)) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  RST_TRY(enqueue_mlp_forward(ctx, B, norm, params, X, logits, choice));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

rst_status rst_mlp_train_step(rst_ctx *ctx, const float *norm, float *params, float *adam_m,
                              float *adam_v, int64_t step, float lr, const float *X,
                              const int32_t *y, const float *w, int64_t B, float *grad,
                              float *loss_host) {
  if (!ctx || !norm || !params || !X || !y || !w || B < 1 || step < 1) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  RST_TRY(ws_reserve(ctx, ws_bytes((size_t)B * kParams, 4) + ws_bytes(B, 4) +
                              ws_bytes(kParams, 4) + ws_bytes(1, 4)));
  float *Gr = ws_take<float>(ctx, (size_t)B * kParams);
  float *loss = ws_take<float>(ctx, B);
  float *g = grad ? grad : ws_take<float>(ctx, kParams);
  float *lm = ws_take<float>(ctx, 1);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)B), dim3(kH), 0, ctx->stream, B, norm, params, X, y,
                     w, Gr, loss);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grad_mean, dim3(grid_for(kParams + 1, kBlock)), dim3(kBlock), 0,
                     ctx->stream, B, Gr, loss, g, lm);
  RST_HIP(hipGetLastError());
  if (adam_m && adam_v && lr > 0.f) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kParams, kBlock)), dim3(kBlock), 0, ctx->stream,
                       params, g, adam_m, adam_v, lr, b1, b2, 1e-8f, bc1, bc2);
    RST_HIP(hipGetLastError());
  }
  if (loss_host) {
    RST_HIP(hipMemcpyAsync(loss_host, lm, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  }
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

rst_status rst_selector_load(rst_ctx *ctx, const void *blob, size_t bytes) {
  if (!ctx || !blob) return RST_E_INVAL;
  const size_t need = 16 + sizeof(float) * (16 + kParams);
  if (bytes != need) return RST_E_INVAL;
  const char *p = static_cast<const char *>(blob);
  if (std::memcmp(p, "RSTSEL01", 8) != 0) return RST_E_INVAL;
  int32_t dims[2];
  std::memcpy(dims, p + 8, 8);
  if (dims[0] != kIn || dims[1] != kH) return RST_E_INVAL;
  const float *vals = reinterpret_cast<const float *>(p + 16);
  for (size_t i = 0; i < 16 + (size_t)kParams; ++i)
    if (!std::isfinite(vals[i])) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  selector_free(ctx);
  Selector *s = new (std::nothrow) Selector();
  if (!s) return RST_E_NOMEM;
  if (hipMalloc(reinterpret_cast<void **>(&s->dev), sizeof(float) * (16 + kParams)) != hipSuccess) {
    delete s;
    return RST_E_NOMEM;
  }
  if (hipMemcpy(s->dev, vals, sizeof(float) * (16 + kParams), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(s->dev);
    delete s;
    return RST_E_DEVICE;
  }
  ctx->selector = s;
  return RST_OK;
}

}  // extern "C"
