// Learned correction policy (a project addition, not in the paper): per-vertex features,
// a small MLP (8 -> 64 -> 64 -> 1, ReLU) that scores each vertex for drift,
// drift labels, and the kernels that train the network. BF16 weights and
// activations, FP32 accumulation on MFMA (v_mfma_f32_16x16x16_bf16), FP32
// master weights trained with Adam.
//
// MFMA 16x16x16 lane layout (wave64, lane l, g = l / 16, c = l % 16):
//   A (16 x 16, rows x k):  lane holds A[c][4g .. 4g+3]
//   B (16 x 16, k x cols):  lane holds B[4g .. 4g+3][c]
//   D (16 x 16, rows x cols): lane holds D[4g .. 4g+3][c]
// A wave processes tiles of 16 samples; layer outputs land in D layout and
// are transposed through LDS when they feed the next layer's A operand.
#include "gg_internal.h"

namespace ggk {

namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float4v mfma(short4v a, short4v b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ short4v pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  short4v v;
  v[0] = (short)a;
  v[1] = (short)b;
  v[2] = (short)c;
  v[3] = (short)d;
  return v;
}

// Inference helpers (16x16x32 bf16 MFMA: lane l holds A[l % 16][k in group
// l / 16] and B[k in group l / 16][l % 16], eight k values per lane).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef short short2v __attribute__((ext_vector_type(2)));
typedef unsigned uint4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4v mfma32(bf16x8 a, bf16x8 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// bf16(relu(a)) | bf16(relu(b)) << 16, round to nearest even (hardware
// conversion); relu on the bfloat16 bits as a signed 16-bit max with 0.
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  const bf16x2 p = __builtin_convertvector((float2v){a, b}, bf16x2);
  const short2v r = __builtin_elementwise_max(__builtin_bit_cast(short2v, p), (short2v){0, 0});
  return __builtin_bit_cast(uint32_t, r);
}

__device__ __forceinline__ bf16x8 bf8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return __builtin_bit_cast(bf16x8, (uint4v){a, b, c, d});
}

// Weights staged in LDS by every block.
struct SW {
  uint16_t w1[16 * 64];  // [k][j], k >= 8 zero
  uint16_t w2[64 * 64];  // [k][j]
  uint16_t w2t[64 * 64]; // [j][k]
  uint16_t w3[64];
  float b1[64], b2[64];
  float b3;
};

__device__ void stage_weights(const MlpDev& w, SW& s) {
  for (int i = threadIdx.x; i < 16 * 64; i += blockDim.x) s.w1[i] = i < 8 * 64 ? w.w1b[i] : (uint16_t)0;
  for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
    const uint16_t v = w.w2b[i];
    s.w2[i] = v;
    s.w2t[(i % 64) * 64 + i / 64] = v;
  }
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    s.w3[i] = w.w3b[i];
    s.b1[i] = w.master[kMlpB1 + i];
    s.b2[i] = w.master[kMlpB2 + i];
  }
  if (threadIdx.x == 0) s.b3 = w.master[kMlpB3];
  __syncthreads();
}

// Forward pass of one 16-sample tile by one wave. feat: bf16 [n][8].
// Produces (in D layout) h1, h2 (bf16 bits, also h1 in LDS [16][64]) and the
// logits of the lane's 4 samples (rows 4g..4g+3).
struct Fwd {
  uint16_t h2[4][4];  // [t][j]: h2[4g+j][16t+c]
  float logit[4];     // samples 4g+j
};

__device__ __forceinline__ void forward_tile(const SW& sw, const uint16_t* feat, int64_t n, int64_t base,
                                             uint16_t* h1s /* LDS [16][64] */, Fwd& F) {
  const int l = __lane_id(), g = l >> 4, c = l & 15;
  // layer 1: A = features of sample base + c, k = 4g..4g+3 (features 0..7, rest 0)
  short4v a1 = pack4(0, 0, 0, 0);
  const int64_t si = base + c;
  if (g < 2 && si < n) {
    const uint16_t* f = feat + si * 8 + 4 * g;
    a1 = pack4(f[0], f[1], f[2], f[3]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int jn = 16 * t + c;
    const short4v b = pack4(sw.w1[(4 * g + 0) * 64 + jn], sw.w1[(4 * g + 1) * 64 + jn], sw.w1[(4 * g + 2) * 64 + jn],
                            sw.w1[(4 * g + 3) * 64 + jn]);
    float4v d = {0.f, 0.f, 0.f, 0.f};
    d = mfma(a1, b, d);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = d[j] + sw.b1[jn];
      h1s[(4 * g + j) * 64 + jn] = f2bf(z > 0.f ? z : 0.f);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  // layer 2: A = h1[c][16s + 4g .. +3]
  float4v d2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) d2[t] = (float4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint16_t* hr = h1s + c * 64 + 16 * s + 4 * g;
    const short4v a = pack4(hr[0], hr[1], hr[2], hr[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int jn = 16 * t + c;
      const uint16_t* wr = sw.w2t + jn * 64 + 16 * s + 4 * g;
      d2[t] = mfma(a, pack4(wr[0], wr[1], wr[2], wr[3]), d2[t]);
    }
  }
  // h2 = bf16(relu(z2)), logit = h2 . w3 + b3 (FP32)
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int jn = 16 * t + c;
    const float w3 = bf2f(sw.w3[jn]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = d2[t][j] + sw.b2[jn];
      const uint16_t h = f2bf(z > 0.f ? z : 0.f);
      F.h2[t][j] = h;
      part[j] += bf2f(h) * w3;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = part[j];
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
    F.logit[j] = v + sw.b3;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Inference: logits (and selection logit > tau when sel is non-null).
// Computed in transposed form: hidden units are the MFMA rows and the 16
// samples of a tile its columns, so the D layout of one layer (lane holds
// units 4g..4g+3 of sample c, g = lane / 16, c = lane % 16) feeds the B
// operand of the next with no LDS round trip. Layers 2 and 3 use 16x16x32
// MFMAs whose k slot j of lane group g stands for hidden unit
//   u(q, g, j) = 32q + 4g + j (j < 4),  32q + 16 + 4g + (j - 4) (j >= 4)
// in k slice q; A (weights) and B (activations) use the same map, so each
// dot product is complete. Layer 3 replicates w3 over the 16 A rows. The
// weights stay in registers for the whole kernel. Each pre-activation is the
// binary32 product sum plus the bias in binary32, as in the reference
// definition, so bfloat16 roundings of the activations agree with it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_forward(
    MlpDev w, const uint16_t* feat, int64_t n, float* logits, uint8_t* sel, float tau, int32_t* sel_count,
    const int32_t* rowptr, unsigned long long* sel_edges) {
  // b1, b2 by units: entry 4t+g holds units 16t+4g .. 16t+4g+3
  __shared__ float4 sb1[16], sb2[16];
  if (threadIdx.x < 64) {
    ((float*)sb1)[threadIdx.x] = w.master[kMlpB1 + threadIdx.x];
    ((float*)sb2)[threadIdx.x] = w.master[kMlpB2 + threadIdx.x];
  }
  const int wv = threadIdx.x >> 6;
  const int l = __lane_id(), g = l >> 4, c = l & 15;
  auto unit = [&](int q, int j) { return 32 * q + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4)); };
  auto pair = [](uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); };
  short4v a1[4];     // [t]: A[row c][k 4g+i] = W1[4g+i][16t+c] (k >= 8 zero)
  bf16x8 a2[4][2];   // [t][q]: A[row c][slot j] = W2[u(q, g, j)][16t+c]
  bf16x8 a3[2];      // [q]: A[any row][slot j] = w3[u(q, g, j)]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) a1[t][i] = g < 2 ? (short)w.w1b[(4 * g + i) * 64 + 16 * t + c] : (short)0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      uint16_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = w.w2b[unit(q, j) * 64 + 16 * t + c];
      a2[t][q] = bf8(pair(e[0], e[1]), pair(e[2], e[3]), pair(e[4], e[5]), pair(e[6], e[7]));
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint16_t e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = w.w3b[unit(q, j)];
    a3[q] = bf8(pair(e[0], e[1]), pair(e[2], e[3]), pair(e[4], e[5]), pair(e[6], e[7]));
  }
  const float b3 = w.master[kMlpB3];
  __syncthreads();
  const int64_t ntiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * 4;
  // B of layer 1 for a tile: features 4g..4g+3 of sample c (k >= 8 and
  // samples past n read as zero); kept two tiles ahead of the compute.
  auto load = [&](int64_t tile) -> uint2 {
    const int64_t si = tile * 16 + c;
    uint2 v = make_uint2(0u, 0u);
    if (tile < ntiles && g < 2 && si < n) v = *(const uint2*)(feat + si * 8 + 4 * g);
    return v;
  };
  int picked = 0;               // selected samples of this lane, over all its tiles
  unsigned long long pe = 0;    // and their in-edges
  int64_t tile = (int64_t)blockIdx.x * 4 + wv;
  uint2 f0 = load(tile), f1 = load(tile + stride);
  for (; tile < ntiles; tile += stride) {
    const uint2 v = f0;
    f0 = f1;
    f1 = load(tile + 2 * stride);
    const short4v x = __builtin_bit_cast(short4v, v);
    // pre-activations: the binary32 product sum, then the bias in binary32
    float4v d1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float4 bb = sb1[4 * t + g];
      d1[t] = mfma(a1[t], x, (float4v){0.f, 0.f, 0.f, 0.f}) + (float4v){bb.x, bb.y, bb.z, bb.w};
    }
    bf16x8 h1[2];  // [q]: B of layer 2
#pragma unroll
    for (int q = 0; q < 2; ++q)
      h1[q] = bf8(relu_bf16x2(d1[2 * q][0], d1[2 * q][1]), relu_bf16x2(d1[2 * q][2], d1[2 * q][3]),
                  relu_bf16x2(d1[2 * q + 1][0], d1[2 * q + 1][1]), relu_bf16x2(d1[2 * q + 1][2], d1[2 * q + 1][3]));
    float4v d2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float4 bb = sb2[4 * t + g];
      d2[t] = mfma32(a2[t][0], h1[0], (float4v){0.f, 0.f, 0.f, 0.f});
      d2[t] = mfma32(a2[t][1], h1[1], d2[t]) + (float4v){bb.x, bb.y, bb.z, bb.w};
    }
    bf16x8 h2[2];  // [q]: B of layer 3
#pragma unroll
    for (int q = 0; q < 2; ++q)
      h2[q] = bf8(relu_bf16x2(d2[2 * q][0], d2[2 * q][1]), relu_bf16x2(d2[2 * q][2], d2[2 * q][3]),
                  relu_bf16x2(d2[2 * q + 1][0], d2[2 * q + 1][1]), relu_bf16x2(d2[2 * q + 1][2], d2[2 * q + 1][3]));
    float4v d3 = mfma32(a3[0], h2[0], (float4v){0.f, 0.f, 0.f, 0.f});
    d3 = mfma32(a3[1], h2[1], d3);
    const int64_t si = tile * 16 + c;
    if (g == 0 && si < n) {
      const float lg = d3[0] + b3;
      if (logits) logits[si] = lg;
      const bool on = lg > tau;
      if (sel) sel[si] = on ? 1 : 0;
      picked += on;
      if (on && rowptr) pe += (unsigned long long)(rowptr[si + 1] - rowptr[si]);
    }
  }
  if (sel_count) {
    // one atomic per block (each)
    __shared__ int wsum[4];
    __shared__ unsigned long long wes[4];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      picked += __shfl_xor(picked, o, 64);
      pe += __shfl_xor(pe, o, 64);
    }
    if (l == 0) {
      wsum[wv] = picked;
      wes[wv] = pe;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
      if (t) atomicAdd(sel_count, t);
      const unsigned long long te = wes[0] + wes[1] + wes[2] + wes[3];
      if (te && sel_edges) atomicAdd(sel_edges, te);
    }
  }
}

// ---------------------------------------------------------------------------
// Training: fused forward + backward of the weighted BCE-with-logits loss
// (mean over the n samples). Each wave writes its partial gradient and loss
// sum to partial[wave][kMlpParams + 1]; k_mlp_reduce adds the waves in order,
// so the result does not depend on timing. The BF16 roundings of h1 / h2 pass
// gradients straight through; ReLU gates on h > 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_grad(MlpDev w, const uint16_t* feat, const float* label, int64_t bn,
                                                  float pos_weight, float* partial) {
  __shared__ SW sw;
  __shared__ uint16_t h1[4][16 * 64];
  __shared__ float dz[4][16 * 64];  // dz2 of the tile, rows = samples
  stage_weights(w, sw);
  const int wv = threadIdx.x >> 6;
  const int l = __lane_id(), g = l >> 4, c = l & 15;
  const float inv_b = 1.0f / (float)bn;
  float4v gw2[4][4];  // [s][t]: dW2[16s + 4g + j][16t + c]
  float4v gw1[4];     // [t]: dW1[4g + j][16t + c] (rows >= 8 unused)
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) gw2[s][t] = (float4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) gw1[t] = (float4v){0.f, 0.f, 0.f, 0.f};
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0};
  float gb3 = 0.f, loss = 0.f;
  const int64_t ntiles = (bn + 15) / 16;
  // the tile's features (16 samples x 8), zero past the end
  __shared__ uint16_t ftile[4][16 * 8];
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    if (l < 16) {
      const int64_t si = tile * 16 + l;
#pragma unroll
      for (int f = 0; f < 8; ++f) ftile[wv][l * 8 + f] = si < bn ? feat[si * 8 + f] : (uint16_t)0;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    Fwd F;
    forward_tile(sw, ftile[wv], 16, 0, h1[wv], F);
    // dlogit for the lane's samples 4g+j
    float dl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t si = tile * 16 + 4 * g + j;
      dl[j] = 0.f;
      if (si < bn) {
        const float y = label[si];
        const float z = F.logit[j];
        const float wt = y > 0.5f ? pos_weight : 1.0f;
        const float p = 1.0f / (1.0f + __expf(-z));
        dl[j] = wt * (p - y) * inv_b;
        if (c == 0) loss += wt * (fmaxf(z, 0.f) - z * y + __logf(1.0f + __expf(-fabsf(z))));
      }
    }
    // dW3, db3, dz2 (D layout) -> LDS transposed copy
    float4v dz2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int jn = 16 * t + c;
      const float w3 = bf2f(sw.w3[jn]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float h = bf2f(F.h2[t][j]);
        gw3[t] += dl[j] * h;
        const float d = h > 0.f ? dl[j] * w3 : 0.f;
        dz2[t][j] = d;
        gb2[t] += d;
        dz[wv][(4 * g + j) * 64 + jn] = d;
      }
    }
    if (c == 0) gb3 += dl[0] + dl[1] + dl[2] + dl[3];
    // dW2[k][jn] += sum_i h1[i][k] dz2[i][jn]: A = h1^T (rows k), B = dz2 (D layout)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 16 * s + c;
      const short4v a = pack4(h1[wv][(4 * g + 0) * 64 + kk], h1[wv][(4 * g + 1) * 64 + kk],
                              h1[wv][(4 * g + 2) * 64 + kk], h1[wv][(4 * g + 3) * 64 + kk]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const short4v b = pack4(f2bf(dz2[t][0]), f2bf(dz2[t][1]), f2bf(dz2[t][2]), f2bf(dz2[t][3]));
        gw2[s][t] = mfma(a, b, gw2[s][t]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // dh1[i][k] = sum_jn dz2[i][jn] W2[k][jn]: A = dz2 rows i (from LDS), B[jn][k] = W2[k][jn]
    float4v dh1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) dh1[t] = (float4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float* dr = dz[wv] + c * 64 + 16 * s + 4 * g;
      const short4v a = pack4(f2bf(dr[0]), f2bf(dr[1]), f2bf(dr[2]), f2bf(dr[3]));
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 16 * t + c;
        const uint16_t* wr = sw.w2 + k * 64 + 16 * s + 4 * g;
        dh1[t] = mfma(a, pack4(wr[0], wr[1], wr[2], wr[3]), dh1[t]);
      }
    }
    // dz1 = dh1 * (h1 > 0); dW1[f][jn] += sum_i x[i][f] dz1[i][jn]
    short4v ax;  // A = x^T: rows f = c (0..7 real), columns samples 4g..4g+3
    {
      const uint16_t* ft = ftile[wv];
      ax = c < 8 ? pack4(ft[(4 * g + 0) * 8 + c], ft[(4 * g + 1) * 8 + c], ft[(4 * g + 2) * 8 + c],
                         ft[(4 * g + 3) * 8 + c])
                 : pack4(0, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int jn = 16 * t + c;
      float4v d1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float h = bf2f(h1[wv][(4 * g + j) * 64 + jn]);
        d1[j] = h > 0.f ? dh1[t][j] : 0.f;
        gb1[t] += d1[j];
      }
      const short4v b = pack4(f2bf(d1[0]), f2bf(d1[1]), f2bf(d1[2]), f2bf(d1[3]));
      gw1[t] = mfma(ax, b, gw1[t]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  // this wave's partial sums: every slot of R is written exactly once
  float* R = partial + ((int64_t)blockIdx.x * 4 + wv) * (kMlpParams + 1);
  // dW2, dW1 (D layout of gw: rows 4g+j within the tile)
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) R[kMlpW2 + (16 * s + 4 * g + j) * 64 + 16 * t + c] = gw2[s][t][j];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * g + j < 8) R[kMlpW1 + (4 * g + j) * 64 + 16 * t + c] = gw1[t][j];
  // vectors reduced over the 4 lane groups g (fixed order)
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float a = gb1[t], b = gb2[t], d = gw3[t];
    a += __shfl_xor(a, 16, 64);
    a += __shfl_xor(a, 32, 64);
    b += __shfl_xor(b, 16, 64);
    b += __shfl_xor(b, 32, 64);
    d += __shfl_xor(d, 16, 64);
    d += __shfl_xor(d, 32, 64);
    if (g == 0) {
      R[kMlpB1 + 16 * t + c] = a;
      R[kMlpB2 + 16 * t + c] = b;
      R[kMlpW3 + 16 * t + c] = d;
    }
  }
  {
    float a = gb3, lo = loss;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      a += __shfl_xor(a, o, 64);
      lo += __shfl_xor(lo, o, 64);
    }
    if (l == 0) {
      R[kMlpB3] = a;
      R[kMlpParams] = lo;
    }
  }
}

// Sums the wave partials: a block takes 32 consecutive slots; lane group j
// (8 groups) adds waves j, j+8, ... in order, then the 8 group sums are added
// in a fixed tree, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* partial, int nwaves, float* grad) {
  __shared__ float red[8][33];
  const int col = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int i = blockIdx.x * 32 + col;
  float a = 0.f;
  if (i < kMlpParams + 1)
    for (int b = grp; b < nwaves; b += 8) a += partial[(int64_t)b * (kMlpParams + 1) + i];
  red[grp][col] = a;
  __syncthreads();
  if (grp == 0 && i < kMlpParams + 1)
    grad[i] = ((red[0][col] + red[1][col]) + (red[2][col] + red[3][col])) +
              ((red[4][col] + red[5][col]) + (red[6][col] + red[7][col]));
}

// Adam on the FP32 master weights, then the BF16 copies.
__global__ void k_mlp_adam(MlpDev w, const float* grad, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) {
    const float gr = grad[i];
    const float m = b1 * w.m[i] + (1.f - b1) * gr;
    const float v = b2 * w.v[i] + (1.f - b2) * gr * gr;
    w.m[i] = m;
    w.v[i] = v;
    const float p = w.master[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    w.master[i] = p;
    if (i < kMlpB1) w.w1b[i - kMlpW1] = f2bf(p);
    else if (i >= kMlpW2 && i < kMlpB2) w.w2b[i - kMlpW2] = f2bf(p);
    else if (i >= kMlpW3 && i < kMlpB3) w.w3b[i - kMlpW3] = f2bf(p);
  }
}

__global__ void k_mlp_sync_bf16(MlpDev w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) {
    const float p = w.master[i];
    if (i < kMlpB1) w.w1b[i - kMlpW1] = f2bf(p);
    else if (i >= kMlpW2 && i < kMlpB2) w.w2b[i - kMlpW2] = f2bf(p);
    else if (i >= kMlpW3 && i < kMlpB3) w.w3b[i - kMlpW3] = f2bf(p);
  }
}

hipError_t launch_mlp_forward(const MlpDev& w, const uint16_t* feat, int64_t n, float* logits, uint8_t* sel, float tau,
                              int32_t* sel_count, const int32_t* rowptr, unsigned long long* sel_edges,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + 3) / 4;
  if (g > 1024) g = 1024;  // 4 waves per SIMD, resident at once; each loads the weights once
  hipLaunchKernelGGL(k_mlp_forward, dim3((int)g), dim3(256), 0, st, w, feat, n, logits, sel, tau, sel_count, rowptr,
                     sel_edges);
  return hipGetLastError();
}

namespace {
int64_t grad_blocks(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + 3) / 4;
  if (g > 256) g = 256;
  return g < 1 ? 1 : g;
}
}  // namespace

int64_t mlp_grad_scratch(int64_t n) { return grad_blocks(n) * 4 * (int64_t)(kMlpParams + 1); }

hipError_t launch_mlp_grad(const MlpDev& w, const uint16_t* feat, const float* label, int64_t n, float pos_weight,
                           float* scratch, float* grad, hipStream_t st) {
  const int64_t nb = grad_blocks(n);
  hipLaunchKernelGGL(k_mlp_grad, dim3((int)nb), dim3(256), 0, st, w, feat, label, n, pos_weight, scratch);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 31) / 32), dim3(256), 0, st, (const float*)scratch,
                     (int)(nb * 4), grad);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDev& w, const float* grad, float lr, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w, grad, lr, 0.9f, 0.999f, 1e-8f,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_sync_bf16(const MlpDev& w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_sync_bf16, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Features: [n][8] bfloat16 rows, word layout (low half first)
//   x: f0 | f1   y: f2 | f3   z: f4 | f5   w: f6 | f7
// f0 = lg(1 + out-degree), f1 = lg(1 + in-degree), f2 = active / in-degree,
// f3, f4 = the last two state deltas, f5..f7 = 0. Every value is computed
// with correctly rounded binary32 operations before its bfloat16 rounding.
// ---------------------------------------------------------------------------
namespace {

// Piecewise-linear base-2 logarithm of y >= 1: L + (y - 2^L) / 2^L.
__device__ __forceinline__ float lg_feat(long long y) {
  const int L = 63 - __clzll(y);
  const float t = __fdiv_rn((float)(y - (1ll << L)), (float)(1ll << L));
  return __fadd_rn((float)L, t);
}

__device__ __forceinline__ float delta_feat(int app, uint32_t now, uint32_t before) {
  if (app == kPR || app == kPPR) {
    const float cn = __uint_as_float(now), co = __uint_as_float(before);
    if (!(cn > 0.0f)) return 0.0f;
    const float r = __fdiv_rn(fabsf(__fsub_rn(cn, co)), cn);
    return r < 1.0f ? r : 1.0f;
  }
  if (app == kSSSP) {
    if (now == kInf) return 0.0f;
    if (before == kInf) return 1.0f;
    if (before == 0u) return 0.0f;
    return __fdiv_rn((float)(before - now), (float)before);
  }
  return now != before ? 1.0f : 0.0f;
}

}  // namespace

__global__ void k_feat_base(int32_t n, const int32_t* rowptr, const int32_t* outdeg, const int32_t* act_cnt,
                            uint16_t* feat) {
  uint4* rows = (uint4*)feat;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t id = rowptr[v + 1] - rowptr[v];
    const int32_t act = act_cnt ? act_cnt[v] : id;
    const float f0 = lg_feat(1ll + outdeg[v]);
    const float f1 = lg_feat(1ll + id);
    const float f2 = id > 0 ? __fdiv_rn((float)act, (float)id) : 0.0f;
    uint4 r = rows[v];
    r.x = (uint32_t)f2bf(f0) | ((uint32_t)f2bf(f1) << 16);
    r.y = (uint32_t)f2bf(f2) | (r.y & 0xFFFF0000u);
    r.z = r.z & 0xFFFFu;
    r.w = 0u;
    rows[v] = r;
  }
}

// f4 <- f3, f3 <- bf16(delta(now, before)).
__global__ void k_feat_shift(int app, int32_t n, const uint32_t* now, const uint32_t* before, uint16_t* feat) {
  uint4* rows = (uint4*)feat;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    uint4 r = rows[v];
    const uint32_t f3 = r.y >> 16;
    const uint32_t d = f2bf(delta_feat(app, now[v], before[v]));
    r.y = (r.y & 0xFFFFu) | (d << 16);
    r.z = (r.z & 0xFFFF0000u) | f3;
    rows[v] = r;
  }
}

// Drift labels of a full superstep: acc = accurate update, apx = the
// approximate update from the same state. PR/PPR (binary32 contributions):
// |acc - apx| > eps * acc; SSSP/CC: acc < apx. label_u8 gets every label,
// label_f the first nf (a trace's free room); audit[0] += positives and
// audit[1] += positives that sel marks; trace_pos += positives among the first nf.
__global__ void k_labels(int app, int32_t n, const uint32_t* acc, const uint32_t* apx, float eps, const uint8_t* sel,
                         uint8_t* label_u8, float* label_f, int32_t nf, unsigned long long* audit,
                         unsigned long long* trace_pos) {
  unsigned long long pos = 0, tp = 0, fpos = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    bool y;
    if (app == kPR || app == kPPR) {
      const float ca = __uint_as_float(acc[v]), cs = __uint_as_float(apx[v]);
      y = fabsf(__fsub_rn(ca, cs)) > __fmul_rn(eps, ca);
    } else {
      y = acc[v] < apx[v];
    }
    if (label_u8) label_u8[v] = y ? 1 : 0;
    if (label_f && v < nf) {
      label_f[v] = y ? 1.0f : 0.0f;
      fpos += y;
    }
    pos += y;
    tp += (y && sel && sel[v]);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    pos += __shfl_xor(pos, o, 64);
    tp += __shfl_xor(tp, o, 64);
    fpos += __shfl_xor(fpos, o, 64);
  }
  __shared__ unsigned long long ws[3][4];
  const int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    ws[0][wv] = pos;
    ws[1][wv] = tp;
    ws[2][wv] = fpos;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pos = ws[0][0] + ws[0][1] + ws[0][2] + ws[0][3];
    tp = ws[1][0] + ws[1][1] + ws[1][2] + ws[1][3];
    fpos = ws[2][0] + ws[2][1] + ws[2][2] + ws[2][3];
    if (audit && pos) atomicAdd(&audit[0], pos);
    if (audit && tp) atomicAdd(&audit[1], tp);
    if (trace_pos && fpos) atomicAdd(trace_pos, fpos);
  }
}

__global__ void k_add_f32(const float* src, float* dst) {
  if (threadIdx.x == 0) *dst += *src;
}

// Clears the flag bits of edge range [b, e) in word k: words wholly inside
// the range are stored, boundary words are masked atomically.
__device__ __forceinline__ void clear_word(uint32_t* bits, int64_t k, int64_t b, int64_t e) {
  const int64_t lo = (b > k * 32 ? b : k * 32) - k * 32;
  const int64_t hi = (e < k * 32 + 32 ? e : k * 32 + 32) - k * 32;
  const uint32_t m = hi - lo >= 32 ? 0xFFFFFFFFu : (((1u << (hi - lo)) - 1u) << lo);
  if (m == 0xFFFFFFFFu) bits[k] = 0u;
  else atomicAnd(&bits[k], ~m);
}

// Clears the flag bits of the listed rows: rows list[0, n_short) one thread
// each (at most a few words), the rest one wave each.
__global__ void k_clear_rows(const int32_t* list, int32_t n_short, int32_t count, const int32_t* rowptr,
                             uint32_t* bits) {
  const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = gtid; t < n_short; t += nthreads) {
    const int u = list[t];
    const int64_t b = rowptr[u], e = rowptr[u + 1];
    if (b < e)
      for (int64_t k = b >> 5; k <= ((e - 1) >> 5); ++k) clear_word(bits, k, b, e);
  }
  const int lane = __lane_id();
  for (int64_t t = n_short + (gtid >> 6); t < count; t += nthreads >> 6) {
    const int u = list[t];
    const int64_t b = rowptr[u], e = rowptr[u + 1];
    if (b >= e) continue;
    for (int64_t k = (b >> 5) + lane; k <= ((e - 1) >> 5); k += 64) clear_word(bits, k, b, e);
  }
}

// Active edges of the selected rows of a partial superstep (the
// approximate gather skips those rows; the superstep reads all their
// in-edges), added to act_sum.
__global__ void k_sel_active(const int32_t* list, int32_t count, const int32_t* act_cnt,
                             unsigned long long* act_sum) {
  unsigned long long a = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    a += (unsigned long long)act_cnt[list[t]];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
  __shared__ unsigned long long wsa[4];
  if (__lane_id() == 0) wsa[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    a = wsa[0] + wsa[1] + wsa[2] + wsa[3];
    if (a) atomicAdd(act_sum, a);
  }
}

static int grid1d(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

hipError_t launch_feat_base(int32_t n, const int32_t* rowptr, const int32_t* outdeg, const int32_t* act_cnt,
                            uint16_t* feat, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_feat_base, dim3(grid1d(n, 256)), dim3(256), 0, st, n, rowptr, outdeg, act_cnt, feat);
  return hipGetLastError();
}

hipError_t launch_feat_shift(int app, int32_t n, const uint32_t* now, const uint32_t* before, uint16_t* feat,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_feat_shift, dim3(grid1d(n, 256)), dim3(256), 0, st, app, n, now, before, feat);
  return hipGetLastError();
}

hipError_t launch_labels(int app, int32_t n, const uint32_t* acc, const uint32_t* apx, float eps, const uint8_t* sel,
                         uint8_t* label_u8, float* label_f, int32_t nf, unsigned long long* audit,
                         unsigned long long* trace_pos, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_labels, dim3(grid1d(n, 4096)), dim3(256), 0, st, app, n, acc, apx, eps, sel, label_u8, label_f,
                     nf, audit, trace_pos);
  return hipGetLastError();
}

hipError_t launch_sel_active(const int32_t* list, int32_t count, const int32_t* act_cnt, unsigned long long* act_sum,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sel_active, dim3(grid1d(count, 4096)), dim3(256), 0, st, list, count, act_cnt, act_sum);
  return hipGetLastError();
}

hipError_t launch_add_f32(const float* src, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_add_f32, dim3(1), dim3(64), 0, st, src, dst);
  return hipGetLastError();
}

hipError_t launch_clear_rows(const int32_t* list, int32_t n_short, int32_t count, const int32_t* rowptr,
                             uint32_t* bits, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t work = (int64_t)n_short + (int64_t)(count - n_short) * 64;
  hipLaunchKernelGGL(k_clear_rows, dim3(grid1d(work, 256)), dim3(256), 0, st, list, n_short, count, rowptr, bits);
  return hipGetLastError();
}

}  // namespace ggk
