// Learned rewrite policy: level features, and the network's forward, backward
// and Adam kernels (FP32). The network is 20 -> 64 -> 64 -> 1 with ReLU and a
// sigmoid output; one wave evaluates one sample with lane j holding hidden unit
// j of both layers, so every reduction is a fixed butterfly or a fixed loop
// (deterministic). Parameters are staged in LDS with padded rows.
#include "common.h"

namespace {

constexpr int NIN = 20, HID = 64, NPAR = 5569;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + HID * NIN, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
static_assert(OFF_B3 + 1 == NPAR, "parameter layout");
constexpr int W1S = NIN + 1, W2S = HID + 1;  // padded LDS row strides
constexpr int kWavesPerBlock = 4;
constexpr int kBwdBlocks = 64;

struct SParams {
  float w1[HID * W1S];
  float b1[HID];
  float w2[HID * W2S];
  float b2[HID];
  float w3[HID];
  float b3;
};

__device__ void load_params(SParams &sp, const float *__restrict__ P) {
  for (int i = threadIdx.x; i < HID * NIN; i += blockDim.x) sp.w1[(i / NIN) * W1S + i % NIN] = P[OFF_W1 + i];
  for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) sp.w2[(i / HID) * W2S + i % HID] = P[OFF_W2 + i];
  for (int i = threadIdx.x; i < HID; i += blockDim.x) {
    sp.b1[i] = P[OFF_B1 + i];
    sp.b2[i] = P[OFF_B2 + i];
    sp.w3[i] = P[OFF_W3 + i];
  }
  if (threadIdx.x == 0) sp.b3 = P[OFF_B3];
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// Forward pass of one sample by one wave. Leaves the normalised features in
// sf, h1 in sh; returns (a1, a2, h2) of this lane's unit and z.
struct Fwd {
  float a1, a2, h2, z;
};

__device__ __forceinline__ Fwd forward_one(const SParams &sp, const float *__restrict__ feat,
                                           const float *__restrict__ norm, int64_t b, float *sf, float *sh) {
  const int j = threadIdx.x & 63;
  if (j < NIN) {
    float f = feat[b * NIN + j];
    if (norm) f = (f - norm[j]) * norm[NIN + j];
    sf[j] = f;
  }
  wsync();
  float a1 = sp.b1[j];
  for (int k = 0; k < NIN; ++k) a1 += sp.w1[j * W1S + k] * sf[k];
  const float h1 = fmaxf(a1, 0.f);
  sh[j] = h1;
  wsync();
  float a2 = sp.b2[j];
  for (int i = 0; i < HID; ++i) a2 += sp.w2[j * W2S + i] * sh[i];
  const float h2 = fmaxf(a2, 0.f);
  const float z = wave_sum(sp.w3[j] * h2) + sp.b3;
  return Fwd{a1, a2, h2, z};
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void k_mlp_forward(const float *__restrict__ P,
                                                                       const float *__restrict__ feat,
                                                                       const float *__restrict__ norm, int32_t B,
                                                                       float *prob) {
  __shared__ SParams sp;
  __shared__ float sf[kWavesPerBlock][NIN], sh[kWavesPerBlock][HID];
  load_params(sp, P);
  __syncthreads();
  const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + w; b < B; b += (int64_t)gridDim.x * kWavesPerBlock) {
    const Fwd f = forward_one(sp, feat, norm, b, sf[w], sh[w]);
    if (j == 0) prob[b] = 1.f / (1.f + expf(-f.z));
    wsync();
  }
}

// Per-wave partial gradients of sum_b w_b BCE_b / B, written to part[wave][*].
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_mlp_backward(
    const float *__restrict__ P, const float *__restrict__ feat, const float *__restrict__ norm,
    const float *__restrict__ label, const float *__restrict__ weight, int32_t B, float *part, float *part_loss) {
  __shared__ SParams sp;
  __shared__ float sf[kWavesPerBlock][NIN], sh[kWavesPerBlock][HID], sd[kWavesPerBlock][HID];
  load_params(sp, P);
  __syncthreads();
  const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
  float gw1[NIN], gw2[HID];
  for (int k = 0; k < NIN; ++k) gw1[k] = 0.f;
  for (int i = 0; i < HID; ++i) gw2[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
  const float invB = 1.f / (float)B;
  for (int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + w; b < B; b += (int64_t)gridDim.x * kWavesPerBlock) {
    const Fwd f = forward_one(sp, feat, norm, b, sf[w], sh[w]);
    const float y = label[b], wt = weight ? weight[b] : 1.f;
    const float p = 1.f / (1.f + expf(-f.z));
    const float dz = wt * (p - y) * invB;
    if (j == 0) {
      loss += wt * (fmaxf(f.z, 0.f) - f.z * y + log1pf(expf(-fabsf(f.z))));
      gb3 += dz;
    }
    gw3 += dz * f.h2;
    const float da2 = f.a2 > 0.f ? dz * sp.w3[j] : 0.f;
    gb2 += da2;
    for (int i = 0; i < HID; ++i) gw2[i] += da2 * sh[w][i];
    sd[w][j] = da2;
    wsync();
    float dh1 = 0.f;
    for (int i = 0; i < HID; ++i) dh1 += sd[w][i] * sp.w2[i * W2S + j];
    const float da1 = f.a1 > 0.f ? dh1 : 0.f;
    gb1 += da1;
    for (int k = 0; k < NIN; ++k) gw1[k] += da1 * sf[w][k];
    wsync();
  }
  float *o = part + ((int64_t)blockIdx.x * kWavesPerBlock + w) * NPAR;
  for (int k = 0; k < NIN; ++k) o[OFF_W1 + j * NIN + k] = gw1[k];
  for (int i = 0; i < HID; ++i) o[OFF_W2 + j * HID + i] = gw2[i];
  o[OFF_B1 + j] = gb1;
  o[OFF_B2 + j] = gb2;
  o[OFF_W3 + j] = gw3;
  if (j == 0) {
    o[OFF_B3] = gb3;
    part_loss[(int64_t)blockIdx.x * kWavesPerBlock + w] = loss * invB;
  }
}

// grad[i] = sum over waves of part[wave][i], in wave order.
__global__ void k_mlp_reduce(const float *__restrict__ part, int32_t nparts, const float *__restrict__ part_loss,
                             float *grad, float *loss) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= NPAR; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    if (i < NPAR) {
      for (int q = 0; q < nparts; ++q) s += part[(int64_t)q * NPAR + i];
      grad[i] = s;
    } else {
      for (int q = 0; q < nparts; ++q) s += part_loss[q];
      *loss = s;
    }
  }
}

__global__ void k_mlp_adam(float *P, const float *__restrict__ g, float *m, float *v, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPAR; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_mlp_mask(const float *__restrict__ prob, int32_t nlev, float thr, uint8_t *mask) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nlev; i += gridDim.x * blockDim.x)
    mask[i] = (i > 0 && prob[i] >= thr) ? 1 : 0;
}

// Tiered actions: a level takes the highest tier whose threshold its
// probability reaches (thresholds ascending) and becomes a source with that
// tier's target budget and fill cap; below the first threshold, and at level
// 0, it is not a source (budget and cap 0: the rewrite's own values).
__global__ void k_mlp_actions(const float *__restrict__ prob, int32_t nlev, MlpTiers t, uint8_t *mask,
                              int32_t *budget, float *cap) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nlev; i += gridDim.x * blockDim.x) {
    int k = -1;
    if (i > 0)
      for (int j = 0; j < t.n; ++j)
        if (prob[i] >= t.thr[j]) k = j;
    mask[i] = k >= 0 ? 1 : 0;
    budget[i] = k >= 0 ? t.budget[k] : 0;
    cap[i] = k >= 0 ? t.cap[k] : 0.0f;
  }
}

// The 20 features of each level (see sptrsv_level_features), from the level
// statistics and the per-row sums of the distance-1 rewrite.
__global__ void k_feat_finalize(int32_t nlev, const int64_t *__restrict__ rows, const int64_t *__restrict__ nnz,
                                const int64_t *__restrict__ cost, double avg, FeatAcc acc, float *feat) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlev; l += (int64_t)gridDim.x * blockDim.x) {
    float *f = feat + l * NIN;
    const int32_t *hist = acc.hist + l * kFeatHist;
    const double R = (double)rows[l];
    f[0] = (float)log1p(R);
    f[1] = (float)log1p((double)nnz[l]);
    f[2] = (float)log1p((double)cost[l]);
    f[3] = (float)(avg > 0.0 ? (double)cost[l] / avg : 0.0);
    f[4] = (float)(R / 32.0);
    f[5] = (float)(R > 0.0 ? (double)nnz[l] / R : 0.0);
    for (int b = 0; b < 6; ++b) f[6 + b] = (float)(R > 0.0 ? (double)hist[b] / R : 0.0);
    f[12] = (float)(nnz[l] > 0 ? (double)acc.sum_lp[l] / (double)nnz[l] : 0.0);
    f[13] = (float)log1p((double)acc.sum_t[l]);
    f[14] = (float)((double)l / (double)nlev);
    f[15] = (float)(l > 0 ? log1p((double)rows[l - 1]) : 0.0);
    f[16] = (float)(R > 0.0 ? (double)hist[6] / R : 0.0);
    f[17] = (float)(R > 0.0 ? (double)hist[7] / R : 0.0);
    f[18] = (float)(R > 0.0 ? log1p((double)acc.sum_span[l] / R) : 0.0);
    f[19] = (float)(R > 0.0 ? (double)hist[8] / R : 0.0);
  }
}

}  // namespace

int mlp_backward_parts() { return kBwdBlocks * kWavesPerBlock; }

hipError_t launch_mlp_forward(const float *P, const float *feat, const float *norm, int32_t B, float *prob,
                              hipStream_t s) {
  if (B <= 0) return hipSuccess;
  int g = (B + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g > 1024 ? 1024 : g;
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(64 * kWavesPerBlock), 0, s, P, feat, norm, B, prob);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *P, const float *feat, const float *norm, const float *label,
                               const float *weight, int32_t B, float *part, float *part_loss, float *grad,
                               float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_backward, dim3(kBwdBlocks), dim3(64 * kWavesPerBlock), 0, s, P, feat, norm, label, weight,
                     B, part, part_loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 256) / 256), dim3(256), 0, s, part, kBwdBlocks * kWavesPerBlock,
                     part_loss, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, float lr, float c1, float c2,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, P, g, m, v, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_mask(const float *prob, int32_t nlev, float thr, uint8_t *mask, hipStream_t s) {
  if (nlev <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_mask, dim3((nlev + 255) / 256), dim3(256), 0, s, prob, nlev, thr, mask);
  return hipGetLastError();
}

hipError_t launch_mlp_actions(const float *prob, int32_t nlev, const MlpTiers &t, uint8_t *mask, int32_t *budget,
                              float *cap, hipStream_t s) {
  if (nlev <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_actions, dim3((nlev + 255) / 256 > 1024 ? 1024 : (nlev + 255) / 256), dim3(256), 0, s,
                     prob, nlev, t, mask, budget, cap);
  return hipGetLastError();
}

hipError_t launch_feat_finalize(int32_t nlev, const int64_t *rows, const int64_t *nnz, const int64_t *cost,
                                double avg, FeatAcc acc, float *feat, hipStream_t s) {
  if (nlev <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_feat_finalize, dim3((nlev + 255) / 256 > 1024 ? 1024 : (nlev + 255) / 256), dim3(256), 0, s,
                     nlev, rows, nnz, cost, avg, acc, feat);
  return hipGetLastError();
}
