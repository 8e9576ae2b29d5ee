// MLP surrogate of the Black-Scholes region (5 -> 64 -> 64 -> 2, GELU in the
// tanh form), used as a further approximation technique: items inside the
// training box are priced by the network, the others by the exact region.
//
//  k_mlp_infer   BF16 MFMA inference with FP32 accumulation.  Every layer is
//                computed transposed (units x items), so the accumulator
//                layout of one layer is, after GELU and conversion, the B
//                operand of the next: the order of the reduction index inside
//                each 32-wide chunk is permuted, and the weights are loaded
//                in the same permuted order.  Items outside the box are
//                ballot-compacted into a queue.
//  k_mlp_fallback the exact region over the queued items.
//  k_mlp_grad    training: forward (FP32 activations, BF16-rounded weights)
//                and backward for 64 items per workgroup of four waves,
//                each wave a quarter of the hidden units; weight-gradient
//                partial sums per workgroup (deterministic, no atomics).
//  k_mlp_adam    sums the partials and applies one Adam step to the FP32
//                master weights.
#include "launch_mlp.hpp"
#include "region_bs.hpp"
#include "wave.hpp"

namespace hpac {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kNH = 64;
constexpr int kOffB1 = 64 * 5, kOffW2 = kOffB1 + 64, kOffB2 = kOffW2 + 64 * 64, kOffW3 = kOffB2 + 64,
              kOffB3 = kOffW3 + 2 * 64, kNumParams = kOffB3 + 2;

// GELU, tanh form: x/2 (1 + tanh(u)) = x / (1 + exp(-2u)),
// u = sqrt(2/pi) (x + 0.044715 x^3); the exponent is formed in base 2.
constexpr float kGeluA = -2.0f * 0.797884560802865356f * 1.44269504088896341f;
constexpr float kGeluB = kGeluA * 0.044715f;
__device__ __forceinline__ float gelu(float x) {
  const float t = x * __builtin_fmaf(x * x, kGeluB, kGeluA);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}
// d/dx of the same function: s + x s (1 - s) (-t'), s = 1/(1 + e^{t}), t' = dt/dx
__device__ __forceinline__ float gelu_d(float x) {
  const float x2 = x * x;
  const float t = x * __builtin_fmaf(x2, kGeluB, kGeluA);
  const float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
  const float dt = __builtin_fmaf(3.0f * kGeluB, x2, kGeluA) * 0.693147180559945309f;
  return s - x * s * (1.0f - s) * dt;
}

__device__ __forceinline__ float round_bf16(float v) { return (float)(__bf16)v; }

// Output o of the network's normalised output yh: the affine map back, then
// exp(v) - shift where the network models log(y + shift).
__device__ __forceinline__ float out_map(const MlpArgs &a, int o, float yh) {
  const float v = __builtin_fmaf(yh, a.out_scale[o], a.out_mean[o]);
  return a.out_shift[o] > 0.0f ? expf(v) - a.out_shift[o] : v;
}

// Training target o in the network's output space.
__device__ __forceinline__ float target_map(const MlpGradArgs &a, int o, float t) {
  return a.out_shift[o] > 0.0f ? logf(t + a.out_shift[o]) : t;
}

// ------------------------------------------------------------------ infer

// permuted position of reduction slot (lane group g, slot j) in chunk c:
// the accumulator rows a lane holds in the two 16-unit tiles of the chunk
__device__ __forceinline__ int kperm(int c, int g, int j) { return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4); }

// Out-of-box item indices are staged per wave in LDS and appended to the
// global queue kQueueStage at a time: one global atomic per wave-flush, not
// one per 64 items (a single counter hit by every wave serialises them).
constexpr int kQueueStage = 256;

__device__ __forceinline__ void queue_flush(const MlpArgs &a, const int32_t *stage, int count, int lane) {
  int base = 0;
  if (lane == 0) base = atomicAdd(a.queue_count, count);
  base = __builtin_amdgcn_readfirstlane(base);
  for (int q = lane; q < count; q += 64) a.queue[base + q] = stage[q];
}

// Persistent: each wave loads the weights into registers once and then walks
// 64-item chunks (chunk = wave id + k * waves in the grid), so the weight
// gather is paid once per wave rather than once per 64 items.
__global__ void __launch_bounds__(256) k_mlp_infer(MlpArgs a) {
  // per wave: the BF16 normalised inputs of its 64 items in the B-operand
  // layout of layer 1 (slots 5..7 zero), and a zero row 64 for lane groups 1..3
  __shared__ bf16x8 xs[4][65];
  __shared__ float ys[4][64][2];  // per wave: the network's normalised outputs
  __shared__ int32_t qstage[4][kQueueStage];
  const int lane = lane_id();
  const int w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;

  // weights in MFMA A layout (lane holds row r of a 16-row tile, reduction
  // slots 8g..8g+7), rounded to BF16
  bf16x8 W1[4], W2[4][2], W3[2];
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      W1[tm][j] = (__bf16)(k < 5 ? a.params[(16 * tm + r) * 5 + k] : 0.0f);
    }
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) W2[tm][c][j] = (__bf16)a.params[kOffW2 + (16 * tm + r) * kNH + kperm(c, g, j)];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) W3[c][j] = (__bf16)(r < 2 ? a.params[kOffW3 + r * kNH + kperm(c, g, j)] : 0.0f);
  // biases in accumulator layout (lane holds rows 4g..4g+3 of each tile)
  floatx4 B1[4], B2[4], B3;
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      B1[tm][j] = a.params[kOffB1 + 16 * tm + 4 * g + j];
      B2[tm][j] = a.params[kOffB2 + 16 * tm + 4 * g + j];
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) B3[j] = (4 * g + j < 2) ? a.params[kOffB3 + 4 * g + j] : 0.0f;

  if (lane == 0) {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    xs[w][64] = z;
  }
  const int64_t chunks = (a.n + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * 4;
  int staged = 0;  // wave-uniform
  // inputs of the wave's next chunk, loaded one chunk ahead
  float xn[5];
  {
    const int64_t i0 = ((int64_t)blockIdx.x * 4 + w) * 64 + lane;
#pragma unroll
    for (int j = 0; j < 5; ++j) xn[j] = i0 < a.n ? a.in[j][i0] : 0.0f;
  }
#pragma unroll 1
  for (int64_t ch = (int64_t)blockIdx.x * 4 + w; ch < chunks; ch += waves) {
    const int64_t i = ch * 64 + lane;
    const bool active = i < a.n;
    // box test, then the loads of the next chunk go out while this one computes
    float x[5];
    bool inside = active;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      x[j] = xn[j];
      inside = inside && x[j] >= a.box_lo[j] && x[j] <= a.box_hi[j];
    }
    if (ch + waves < chunks) {  // wave-uniform
      const int64_t inx = i + waves * 64;
#pragma unroll
      for (int j = 0; j < 5; ++j) xn[j] = inx < a.n ? a.in[j][inx] : 0.0f;
    }
    const uint64_t out_mask = ballot(active && !inside);
    // the previous chunk's LDS reads are done before anything is rewritten
    wave_lds_fence();
    if (out_mask) {
      const int cnt = popc(out_mask);
      if (staged + cnt > kQueueStage) {
        queue_flush(a, qstage[w], staged, lane);
        staged = 0;
        wave_lds_fence();
      }
      if (active && !inside) qstage[w][staged + popc(out_mask & ((1ull << lane) - 1))] = (int32_t)i;
      staged += cnt;
    }
    float xh[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) xh[j] = (x[j] - a.in_center[j]) * a.in_scale[j];
    {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (__bf16)(j < 5 ? xh[j < 5 ? j : 0] : 0.0f);
      xs[w][lane] = v;
    }
    wave_lds_fence();

#pragma unroll 2
    for (int tn = 0; tn < 4; ++tn) {
      // B operand of layer 1: inputs of item 16 tn + r in slots 0..7 of lane
      // group 0, zeros elsewhere
      const bf16x8 xb = xs[w][g == 0 ? 16 * tn + r : 64];
      floatx4 D1[4];
#pragma unroll
      for (int tm = 0; tm < 4; ++tm) D1[tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W1[tm], xb, B1[tm], 0, 0, 0);
      // GELU, BF16, and the permuted B operand of layer 2: chunk c, slot j
      bf16x8 h1[2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) h1[c][j] = (__bf16)gelu(D1[2 * c + (j >> 2)][j & 3]);
      floatx4 D2[4];
#pragma unroll
      for (int tm = 0; tm < 4; ++tm) {
        D2[tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W2[tm][0], h1[0], B2[tm], 0, 0, 0);
        D2[tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W2[tm][1], h1[1], D2[tm], 0, 0, 0);
      }
      bf16x8 h2[2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) h2[c][j] = (__bf16)gelu(D2[2 * c + (j >> 2)][j & 3]);
      floatx4 D3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W3[0], h2[0], B3, 0, 0, 0);
      D3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W3[1], h2[1], D3, 0, 0, 0);
      // rows 0 and 1 (the two outputs) live in lanes 0..15, slots 0 and 1
      if (g == 0) {
        ys[w][16 * tn + r][0] = D3[0];
        ys[w][16 * tn + r][1] = D3[1];
      }
    }
    wave_lds_fence();
    if (active && inside) {
      // the output map once per item, each lane on its own item
      a.out[0][i] = out_map(a, 0, ys[w][lane][0]);
      a.out[1][i] = out_map(a, 1, ys[w][lane][1]);
    }
  }
  if (staged > 0) {
    wave_lds_fence();
    queue_flush(a, qstage[w], staged, lane);
  }
}

__global__ void __launch_bounds__(256) k_mlp_fallback(MlpArgs a) {
  const int count = *a.queue_count;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < count; q += gridDim.x * blockDim.x) {
    const int64_t i = a.queue[q];
    float x[5], y[2];
#pragma unroll
    for (int j = 0; j < 5; ++j) x[j] = a.in[j][i];
    RegionBSPrice::eval(x, y);
    a.out[0][i] = y[0];
    a.out[1][i] = y[1];
  }
}

__global__ void k_zero_int(int32_t *p) { *p = 0; }

// ------------------------------------------------------------------ train

// 64 items per workgroup, one per lane of each of its four waves; wave w
// computes hidden units 16w..16w+15 of each layer (the full layers meet in
// LDS), so the work of one item is spread over four SIMDs.  Every value is
// formed in the same order as by a single lane computing the whole item:
// each wave forms the network's output itself from the LDS copy of the
// second hidden layer.
__global__ void __launch_bounds__(256) k_mlp_grad(MlpGradArgs a) {
  __shared__ float W[kNumParams];           // BF16-rounded weights, FP32 biases
  __shared__ float h1s[64][kNH + 1], h2s[64][kNH + 1], dz2s[64][kNH + 1], dz1s[64][kNH + 1];
  __shared__ float xhs[64][5], dys[64][2], errs[64];
  const int T = threadIdx.x;
  const int w = T >> 6, t = T & 63;  // wave, and the lane's item in the workgroup
  const int u0 = 16 * w;             // the wave's hidden units
  for (int p = T; p < kNumParams; p += 256) {
    const bool is_bias = (p >= kOffB1 && p < kOffW2) || (p >= kOffB2 && p < kOffW3) || p >= kOffB3;
    W[p] = is_bias ? a.params[p] : round_bf16(a.params[p]);
  }
  const int64_t i = (int64_t)blockIdx.x * 64 + t;
  const bool active = i < a.n;
  float xh[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) xh[j] = active ? (a.x[j][i] - a.in_center[j]) * a.in_scale[j] : 0.0f;
  if (w == 0) {
#pragma unroll
    for (int j = 0; j < 5; ++j) xhs[t][j] = xh[j];
  }
  __syncthreads();
  // forward, layer 1: the wave's units
  float z1[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int o = u0 + u;
    float z = W[kOffB1 + o];
#pragma unroll
    for (int j = 0; j < 5; ++j) z = __builtin_fmaf(W[o * 5 + j], xh[j], z);
    z1[u] = z;
    h1s[t][o] = gelu(z);
  }
  __syncthreads();
  // layer 2: the wave's units, from the whole first layer
  float z2[16];
  {
    float h[kNH];
#pragma unroll
    for (int j = 0; j < kNH; ++j) h[j] = h1s[t][j];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int o = u0 + u;
      float z = W[kOffB2 + o];
#pragma unroll
      for (int j = 0; j < kNH; ++j) z = __builtin_fmaf(W[kOffW2 + o * kNH + j], h[j], z);
      z2[u] = z;
      h2s[t][o] = gelu(z);
    }
  }
  __syncthreads();
  // layer 3, in every wave, from the whole second layer
  float yh0 = W[kOffB3], yh1 = W[kOffB3 + 1];
#pragma unroll 8
  for (int j = 0; j < kNH; ++j) {
    const float h = h2s[t][j];
    yh0 = __builtin_fmaf(W[kOffW3 + j], h, yh0);
    yh1 = __builtin_fmaf(W[kOffW3 + kNH + j], h, yh1);
  }
  // loss 1/(2N) sum (yh - th)^2 over the N training items and both outputs
  const float e0 = active ? yh0 - (target_map(a, 0, a.t[0][i]) - a.out_mean[0]) / a.out_scale[0] : 0.0f;
  const float e1 = active ? yh1 - (target_map(a, 1, a.t[1][i]) - a.out_mean[1]) / a.out_scale[1] : 0.0f;
  const float dy0 = e0 * a.inv_count, dy1 = e1 * a.inv_count;
  if (w == 0) {
    dys[t][0] = dy0;
    dys[t][1] = dy1;
    errs[t] = e0 * e0 + e1 * e1;
  }
  // backward through layer 3 and the second GELU: the wave's units
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int j = u0 + u;
    const float dh = W[kOffW3 + j] * dy0 + W[kOffW3 + kNH + j] * dy1;
    dz2s[t][j] = dh * gelu_d(z2[u]);
  }
  __syncthreads();
  // through layer 2 and the first GELU: the wave's units, from all of dz2
  {
    float d2[kNH];
#pragma unroll
    for (int o = 0; o < kNH; ++o) d2[o] = dz2s[t][o];
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      const int j = u0 + u;
      float dh = 0.0f;
#pragma unroll
      for (int o = 0; o < kNH; ++o) dh = __builtin_fmaf(W[kOffW2 + o * kNH + j], d2[o], dh);
      dz1s[t][j] = dh * gelu_d(z1[u]);
    }
  }
  __syncthreads();
  // per-workgroup weight gradients, each summed over the 64 items in order
  float *part = a.grad_partials + (int64_t)blockIdx.x * kNumParams;
  {
    // layer 2: thread T owns output unit T / 4, input units 16 (T % 4) ..
    const int o = T >> 2, j0 = 16 * (T & 3);
    float acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
    for (int it = 0; it < 64; ++it) {
      const float d2 = dz2s[it][o];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = __builtin_fmaf(d2, h1s[it][j0 + q], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) part[kOffW2 + o * kNH + j0 + q] = acc[q];
  }
  if (w == 0) {
    // layer 1 and the first two biases: lane t owns unit t
    float gb1 = 0.0f, gw1[5] = {0, 0, 0, 0, 0};
    float gb2 = 0.0f;
    for (int it = 0; it < 64; ++it) {
      const float d1 = dz1s[it][t];
      gb1 += d1;
#pragma unroll
      for (int k = 0; k < 5; ++k) gw1[k] = __builtin_fmaf(d1, xhs[it][k], gw1[k]);
      gb2 += dz2s[it][t];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) part[t * 5 + k] = gw1[k];
    part[kOffB1 + t] = gb1;
    part[kOffB2 + t] = gb2;
  } else if (w == 1) {
    // layer 3: 2 x 64 weights; lane t owns input unit t
    float g0 = 0.0f, g1 = 0.0f;
    for (int it = 0; it < 64; ++it) {
      g0 = __builtin_fmaf(dys[it][0], h2s[it][t], g0);
      g1 = __builtin_fmaf(dys[it][1], h2s[it][t], g1);
    }
    part[kOffW3 + t] = g0;
    part[kOffW3 + kNH + t] = g1;
  } else if (w == 2) {
    if (t < 2) {
      float s = 0.0f;
      for (int it = 0; it < 64; ++it) s += dys[it][t];
      part[kOffB3 + t] = s;
    } else if (t == 2) {
      float s = 0.0f;
      for (int it = 0; it < 64; ++it) s += errs[it];
      a.loss_partials[blockIdx.x] = s;
    }
  }
}

__global__ void __launch_bounds__(256) k_mlp_adam(AdamArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNumParams) return;
  // the partials summed in workgroup order; sixteen loads in flight at a
  // time instead of one memory latency per partial
  constexpr int kU = 16;
  float g = 0.0f;
  for (int64_t b0 = 0; b0 < a.blocks; b0 += kU) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = b0 + u < a.blocks ? a.grad_partials[(b0 + u) * kNumParams + p] : 0.0f;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (b0 + u < a.blocks) g += v[u];
  }
  const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * g * g;
  a.m[p] = m;
  a.v[p] = v;
  const float mh = m / a.bc1, vh = v / a.bc2;
  a.params[p] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

// --------------------------------------------------------------- launchers

int mlp_num_params() { return kNumParams; }

hipError_t launch_mlp_infer(const MlpArgs &a, hipStream_t stream) {
  // one resident wave per SIMD slot the kernel's register use allows
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_infer, 256, 0);
  if (e != hipSuccess) return e;
  const int64_t want = (a.n + 255) / 256;
  const int64_t resident = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  const unsigned grid = (unsigned)(want < resident ? (want < 1 ? 1 : want) : resident);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, stream, a.queue_count);
  hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, stream, a);
  int blocks = (int)((a.n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_mlp_fallback, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpGradArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((a.n + 63) / 64)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const AdamArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNumParams + 255) / 256), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace hpac
