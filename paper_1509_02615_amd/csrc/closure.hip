// Learned coarse closure: a per-node network on stencil-gathered fields that
// corrects a coarse Navier-Stokes right-hand side (trained on fine runs of
// the same method restricted to the coarse nodes).
//
// Network: x (148 gathered values + 1 node value, padded to 160) ->
// h1 = tanh(W1 x + b1) (128) -> h2 = tanh(W2 h1 + b2) (128) -> y = W3 h2 + b3
// (4, padded to 16). BF16 weights and activations, FP32 accumulation on the
// matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Every product is one kernel, C = A . B^T with both operands contiguous
// along the contraction index (samples x features, or features x samples
// for the weight gradients), and an epilogue per use:
//   bias + activation -> BF16  (hidden layers)
//   bias -> FP32               (output layer)
//   x a'(h) -> BF16            (back-propagation through the activation)
//   atomic FP32 accumulation   (weight gradients, split over sample chunks)
// Lane layout of the 16x16x32 instruction: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16] (so row l%16 of B^T) and D[4(l/16)..+3][l%16].
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "model.hpp"

namespace {

constexpr int HID = 128, KIN = 160, NOUT = 16, NSLOT_MAX = 37;
constexpr int OW1 = 0, OB1 = OW1 + HID * KIN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + NOUT * HID, NPARAM = OB3 + NOUT;
static_assert(NPARAM == RBFFD_CLOSURE_NPARAMS, "parameter layout");

typedef __attribute__((ext_vector_type(4))) float f4v;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8v;

enum { EPI_ACT = 0, EPI_BIAS = 1, EPI_DACT = 2, EPI_ATOMIC = 3 };

// C[m][n] (epilogue) = sum_k A[m][k] B[n][k]; A: M x K (lda), B: 16*NT x K
// (ldb); K a multiple of 32 within [kbeg, kend) = blockIdx.y's chunk. Four
// wavefronts, each 16 rows x 16*NT columns.
template <int EPI, int NT>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const __bf16 *__restrict__ A, int lda,
                                                      const __bf16 *__restrict__ B, int ldb, int M, int K,
                                                      int k_chunk, const float *__restrict__ bias,
                                                      const __bf16 *__restrict__ H, int ldh, void *C, int ldc,
                                                      int act) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 64 + wave * 16;
  const int kbeg = blockIdx.y * k_chunk, kend = min(K, kbeg + k_chunk);
  f4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  const int row = m0 + (lane & 15), koff = 8 * (lane >> 4);
  const bool rowok = row < M;
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    bf8v a;
    if (rowok) {
      a = *reinterpret_cast<const bf8v *>(A + static_cast<int64_t>(row) * lda + k0 + koff);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = static_cast<__bf16>(0.0f);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf8v b = *reinterpret_cast<const bf8v *>(B + static_cast<int64_t>(16 * t + (lane & 15)) * ldb + k0 + koff);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = 16 * t + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = m0 + 4 * (lane >> 4) + i;
      if (r >= M) continue;
      const float v = acc[t][i];
      const int64_t o = static_cast<int64_t>(r) * ldc + c;
      if constexpr (EPI == EPI_ACT) {
        const float z = v + bias[c];
        static_cast<__bf16 *>(C)[o] =
            static_cast<__bf16>(act == RBFFD_ACT_RELU ? __builtin_elementwise_maximum(z, 0.0f) : tanhf(z));
      } else if constexpr (EPI == EPI_BIAS) {
        static_cast<float *>(C)[o] = v + bias[c];
      } else if constexpr (EPI == EPI_DACT) {
        const float h = static_cast<float>(H[static_cast<int64_t>(r) * ldh + c]);
        static_cast<__bf16 *>(C)[o] = static_cast<__bf16>(act == RBFFD_ACT_RELU ? (h > 0.0f ? v : 0.0f)
                                                                                : v * (1.0f - h * h));
      } else {
        atomicAdd(static_cast<float *>(C) + o, v);
      }
    }
  }
}

// ---- fused forward pass -------------------------------------------------
// One kernel from the state to the normalised correction. The products are
// computed transposed, H^T = W X^T: the weights are the A operand (packed in
// LDS as per-lane fragments, shared by every sample tile of the block) and
// the samples the B operand, so lane l always holds sample l%16 of its tile:
// the input fragment is gathered straight from the state, and a layer's
// accumulators (outputs 16t + 4(l/16) + i) become the next layer's B
// fragment without moving data between lanes, once the contraction index of
// the next weight matrix is permuted to that order (mlp_perm). The biases
// enter as the accumulator input of each output tile's first product.
constexpr int FR1 = 8 * 5, FR2 = 8 * 4, FR3 = 4, NFRAG = FR1 + FR2 + FR3;  // 16 B x 64 lanes each
constexpr int NBIAS = HID + HID + NOUT;
constexpr size_t MLP_LDS = static_cast<size_t>(NFRAG) * 64 * 16 + NBIAS * sizeof(float);

// Position p of a 32-wide contraction block j of layers 2 and 3 -> hidden unit.
__host__ __device__ constexpr int mlp_perm(int j, int p) {
  return 32 * j + ((p & 7) < 4 ? 4 * (p >> 3) + (p & 7) : 16 + 4 * (p >> 3) + (p & 7) - 4);
}

// frag[f][lane][q], f < FR1: W1 tile (t = f / 5, k-block j = f % 5); then W2
// tiles (t = f' / 4, j = f' % 4) and W3 (j) with permuted contraction index.
__global__ void frag_pack_kernel(const float *__restrict__ p, __bf16 *__restrict__ frag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NFRAG * 512) return;
  const int f = t >> 9, l = (t >> 3) & 63, q = t & 7;
  const int row = l & 15, pos = 8 * (l >> 4) + q;
  float v;
  if (f < FR1) {
    v = p[OW1 + (16 * (f / 5) + row) * KIN + 32 * (f % 5) + pos];
  } else if (f < FR1 + FR2) {
    const int g = f - FR1;
    v = p[OW2 + (16 * (g / 4) + row) * HID + mlp_perm(g % 4, pos)];
  } else {
    v = p[OW3 + row * HID + mlp_perm(f - FR1 - FR2, pos)];
  }
  frag[t] = static_cast<__bf16>(v);
}

// The activation; relu propagates NaN (IEEE maximum, one instruction).
template <int ACT> __device__ __forceinline__ float act_fn(float v) {
  if constexpr (ACT == RBFFD_ACT_RELU) {
    return __builtin_elementwise_maximum(v, 0.0f);
  } else {
    return tanhf(v);
  }
}

// Input fragment of contraction block j for one sample: slots 8j + 2g and
// 8j + 2g + 1 (four fields each). Branch-free: a slot past the stencil
// re-reads the node itself (difference 0); slot 37 carries the node value.
__device__ __forceinline__ bf8v gather_block(const float *__restrict__ y, const int *__restrict__ idx_t, int64_t Na,
                                             int n, int E, float nodev, float4 inv, int64_t i, int e, float4 own,
                                             int slot0) {
  bf8v x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int slot = slot0 + h;
    const int64_t j = (slot >= 1 && slot < n) ? idx_t[static_cast<int64_t>(slot) * Na + i] : i;
    const float4 f = *reinterpret_cast<const float4 *>(y + (j * E + e) * 4);
    const float4 b = slot == 0 ? make_float4(0.f, 0.f, 0.f, 0.f) : own;
    float v0 = (f.x - b.x) * inv.x, v1 = (f.y - b.y) * inv.y, v2 = (f.z - b.z) * inv.z, v3 = (f.w - b.w) * inv.w;
    if (slot == NSLOT_MAX) v0 = nodev;
    x[4 * h + 0] = static_cast<__bf16>(v0);
    x[4 * h + 1] = static_cast<__bf16>(v1);
    x[4 * h + 2] = static_cast<__bf16>(v2);
    x[4 * h + 3] = static_cast<__bf16>(v3);
  }
  return x;
}

// Y[s][0..3] for S samples, T tiles of 16 samples per wavefront; blocks of
// W wavefronts share one LDS copy of the weights and loop over contiguous
// unit ranges (XCD-aware block order); OCC wavefronts per SIMD bound the
// registers. The launch shapes (T, W, OCC) rbffd_closure_tune chooses from
// are kMlpShapes; a sample's arithmetic is the same in every shape. Measured
// on 557,056 samples: one 16-wavefront block per compute unit at four
// wavefronts per SIMD and T = 1 is fastest (more wavefronts hide the gather
// latency better than larger tiles save LDS reads of the weight fragments).
template <int T, int MLP_WAVES, int MLP_OCC, int ACT>
__global__ __launch_bounds__(64 * MLP_WAVES) __attribute__((amdgpu_waves_per_eu(MLP_OCC, MLP_OCC))) void
mlp_forward_kernel(
    const float *__restrict__ y, const int *__restrict__ idx_t, int64_t Na, int n, int E,
    const float *__restrict__ nodef, float4 inv, const __bf16 *__restrict__ frag_g, const float *__restrict__ params,
    float *__restrict__ Y, int64_t S) {
  extern __shared__ __attribute__((aligned(16))) unsigned char mlp_lds[];
  const bf8v *s_frag = reinterpret_cast<const bf8v *>(mlp_lds);
  float *s_bias = reinterpret_cast<float *>(mlp_lds + static_cast<size_t>(NFRAG) * 64 * 16);
  {
    const f4v *src = reinterpret_cast<const f4v *>(frag_g);
    f4v *dst = reinterpret_cast<f4v *>(mlp_lds);
    for (int k = threadIdx.x; k < NFRAG * 64; k += 64 * MLP_WAVES) dst[k] = src[k];
    for (int k = threadIdx.x; k < NBIAS; k += 64 * MLP_WAVES)
      s_bias[k] = k < HID ? params[OB1 + k] : (k < 2 * HID ? params[OB2 + k - HID] : params[OB3 + k - 2 * HID]);
  }
  __syncthreads();
  const f4v *s_b4 = reinterpret_cast<const f4v *>(s_bias);   // 4 consecutive biases per lane group
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int64_t units = (S + 16 * T - 1) / (16 * T);
  const int64_t nb = gridDim.x, b = blockIdx.x, full = (nb / 8) * 8;
  const int64_t lb = b >= full ? b : (b % 8) * (nb / 8) + b / 8;
  const int64_t per = (units + nb - 1) / nb;
  const int64_t u_end = min(units, (lb + 1) * per);
  for (int64_t u = lb * per + wave; u < u_end; u += MLP_WAVES) {
    const int64_t base = u * 16 * T;
    // keeps the weight fragments' LDS reads inside the loop: hoisted out of
    // it as loop-invariant they would need 304 registers
    asm volatile("" ::: "memory");
    int64_t si[T];
    int se[T];
    float4 own[T];
    float nodev[T];
#pragma unroll
    for (int tl = 0; tl < T; ++tl) {
      const int64_t s = min(base + 16 * tl + r, S - 1);     // rows past S compute a copy, never stored
      si[tl] = s / E;
      se[tl] = static_cast<int>(s - si[tl] * E);
      own[tl] = *reinterpret_cast<const float4 *>(y + s * 4);
      nodev[tl] = nodef[si[tl]];
    }
    // output tile outermost: only one tile's accumulators are live, so the
    // whole input (5 blocks) and both hidden fragments fit in 128 registers
    // and four wavefronts run per SIMD
    bf8v x[5][T];
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
      for (int tl = 0; tl < T; ++tl)
        x[j][tl] = gather_block(y, idx_t, Na, n, E, nodev[tl], inv, si[tl], se[tl], own[tl], 8 * j + 2 * g);
    bf8v hb[4][T];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      f4v acc[T];
      const f4v c0 = s_b4[4 * t + g];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const bf8v a = s_frag[(t * 5 + j) * 64 + lane];
#pragma unroll
        for (int tl = 0; tl < T; ++tl)
          acc[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, x[j][tl], j == 0 ? c0 : acc[tl], 0, 0, 0);
      }
#pragma unroll
      for (int tl = 0; tl < T; ++tl)
#pragma unroll
        for (int i = 0; i < 4; ++i) hb[t >> 1][tl][4 * (t & 1) + i] = static_cast<__bf16>(act_fn<ACT>(acc[tl][i]));
    }
    bf8v hb2[4][T];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      f4v acc[T];
      const f4v c0 = s_b4[32 + 4 * t + g];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf8v a = s_frag[FR1 * 64 + (t * 4 + j) * 64 + lane];
#pragma unroll
        for (int tl = 0; tl < T; ++tl)
          acc[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[j][tl], j == 0 ? c0 : acc[tl], 0, 0, 0);
      }
#pragma unroll
      for (int tl = 0; tl < T; ++tl)
#pragma unroll
        for (int i = 0; i < 4; ++i) hb2[t >> 1][tl][4 * (t & 1) + i] = static_cast<__bf16>(act_fn<ACT>(acc[tl][i]));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int tl = 0; tl < T; ++tl) hb[j][tl] = hb2[j][tl];
    // layer 3: one output tile, outputs 0..3 in the lanes of group 0
    f4v out[T];
    const f4v c3 = s_b4[64 + g];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf8v a = s_frag[(FR1 + FR2 + j) * 64 + lane];
#pragma unroll
      for (int tl = 0; tl < T; ++tl)
        out[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[j][tl], j == 0 ? c3 : out[tl], 0, 0, 0);
    }
    if (g == 0) {
#pragma unroll
      for (int tl = 0; tl < T; ++tl) {
        const int64_t s = base + 16 * tl + r;
        if (s < S) *reinterpret_cast<float4 *>(Y + s * 4) = make_float4(out[tl][0], out[tl][1], out[tl][2], out[tl][3]);
      }
    }
  }
}

// Matrix-core throughput probe: every wavefront runs `iters` rounds of four
// independent BF16 products on register operands (no memory traffic), of
// shape 16x16x32 (SHAPE 0) or 32x32x16 (SHAPE 1); each lane stores one sum so
// that none of them is dead.
template <int SHAPE> __global__ __launch_bounds__(256) void mfma_probe_kernel(float *__restrict__ out, int iters) {
  typedef __attribute__((ext_vector_type(16))) float f16v;
  const int tid = threadIdx.x;
  bf8v a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = static_cast<__bf16>(1.0f + 0.001f * static_cast<float>((tid + q) & 7));
    b[q] = static_cast<__bf16>(0.5f - 0.001f * static_cast<float>((tid * 3 + q) & 7));
  }
  float v = 0.0f;
  if constexpr (SHAPE == 0) {
    f4v acc[4] = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) v += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  } else {
    f16v acc[4] = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) v += acc[u][0] + acc[u][5] + acc[u][10] + acc[u][15];
  }
  out[static_cast<int64_t>(blockIdx.x) * 256 + tid] = v;
}

// Input features, one thread per (sample, 4-value group): slot 0 = own
// fields, slots 1..36 = differences, group 37 = node value + zeros, 38..39 = 0.
__global__ void features_kernel(const float *__restrict__ y, const int *__restrict__ idx_t, int64_t Na, int n, int E,
                                const float *__restrict__ nodef, float4 inv_scale, __bf16 *__restrict__ X) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t S = Na * E;
  if (t >= S * 40) return;
  const int64_t s = t / 40;
  const int k = static_cast<int>(t - s * 40);
  const int64_t i = s / E;
  const int e = static_cast<int>(s - i * E);
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  const float4 own = *reinterpret_cast<const float4 *>(y + (i * E + e) * 4);
  if (k == 0) {
    v[0] = own.x * inv_scale.x;
    v[1] = own.y * inv_scale.y;
    v[2] = own.z * inv_scale.z;
    v[3] = own.w * inv_scale.w;
  } else if (k < n) {
    const int j = idx_t[static_cast<int64_t>(k) * Na + i];
    const float4 f = *reinterpret_cast<const float4 *>(y + (static_cast<int64_t>(j) * E + e) * 4);
    v[0] = (f.x - own.x) * inv_scale.x;
    v[1] = (f.y - own.y) * inv_scale.y;
    v[2] = (f.z - own.z) * inv_scale.z;
    v[3] = (f.w - own.w) * inv_scale.w;
  } else if (k == NSLOT_MAX) {
    v[0] = nodef[i];
  }
  __bf16 *o = X + s * KIN + 4 * k;
  for (int c = 0; c < 4; ++c) o[c] = static_cast<__bf16>(v[c]);
}

// out[c][s] = in[s][c] for s < S, 0 for S <= s < Sp (Cn, ldi and Sp multiples
// of 8); 64x64 tiles through LDS, with 16-byte loads along c and 16-byte
// stores along s.
__global__ __launch_bounds__(256) void transpose_kernel(const __bf16 *__restrict__ in, int ldi, int64_t S, int Cn,
                                                        __bf16 *__restrict__ out, int64_t Sp) {
  __shared__ __attribute__((aligned(16))) __bf16 tile[64][72];  // [s][c]; 144-byte rows
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int c0 = blockIdx.y * 64;
  for (int v = threadIdx.x; v < 512; v += 256) {  // 64 rows x 8 vectors of 8
    const int r = v >> 3, cv = (v & 7) * 8;
    const int64_t s = s0 + r;
    const int c = c0 + cv;
    bf8v x;
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = static_cast<__bf16>(0.0f);
    if (s < S && c < Cn) x = *reinterpret_cast<const bf8v *>(in + s * ldi + c);
    *reinterpret_cast<bf8v *>(&tile[r][cv]) = x;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < 512; v += 256) {  // 64 columns x 8 vectors of 8 samples
    const int cr = v >> 3, sv = (v & 7) * 8;
    const int c = c0 + cr;
    const int64_t s = s0 + sv;
    if (c < Cn && s < Sp) {
      bf8v y;
#pragma unroll
      for (int q = 0; q < 8; ++q) y[q] = tile[sv + q][cr];
      *reinterpret_cast<bf8v *>(out + static_cast<int64_t>(c) * Sp + s) = y;
    }
  }
}

// dY = 2 (Y - T) / (4 S) for the 4 outputs (BF16, padded to 32 columns for
// the next product; FP32 copy [S][4] for the output bias gradient) and the
// loss sum of (Y - T)^2 / (4 S).
__global__ void loss_kernel(const float *__restrict__ Y, const float *__restrict__ T, int64_t S,
                            __bf16 *__restrict__ dY, float *__restrict__ dY32, double *__restrict__ loss) {
  __shared__ double red[256];
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (s < S) {
    const float inv = 1.0f / static_cast<float>(4 * S);
    for (int c = 0; c < 32; ++c) {
      float g = 0.0f;
      if (c < 4) {
        const float d = Y[s * NOUT + c] - T[s * 4 + c];
        l += static_cast<double>(d) * d;
        g = 2.0f * d * inv;
        dY32[s * 4 + c] = g;
      }
      dY[s * 32 + c] = static_cast<__bf16>(g);
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (4.0 * static_cast<double>(S)));
}

// grad[c] += sum_s D[s][c] over a chunk of samples (bias gradients). A block
// is COLSUM_SLICES x 128 threads: each column's chunk is summed in that many
// interleaved slices (independent loads in flight), the slices are added in
// LDS, and one atomic per column and block goes to grad.
constexpr int COLSUM_SLICES = 8;
template <class T>
__global__ __launch_bounds__(128 * COLSUM_SLICES) void colsum_kernel(const T *__restrict__ D, int ldd, int64_t S,
                                                                    int Cn, int64_t chunk, float *__restrict__ grad) {
  __shared__ float part[COLSUM_SLICES][128];
  const int c = static_cast<int>(threadIdx.x) & 127, sl = static_cast<int>(threadIdx.x) >> 7;
  float acc = 0.0f;
  if (c < Cn) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * chunk, e = min(S, b + chunk);
#pragma unroll 8
    for (int64_t s = b + sl; s < e; s += COLSUM_SLICES) acc += static_cast<float>(D[s * ldd + c]);
  }
  part[sl][c] = acc;
  __syncthreads();
  if (sl == 0 && c < Cn) {
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < COLSUM_SLICES; ++q) t += part[q][c];
    atomicAdd(grad + c, t);
  }
}

// BF16 copies of the weights (and the transposed W2, W3 the backward pass uses).
__global__ void pack_kernel(const float *__restrict__ p, __bf16 *__restrict__ w1, __bf16 *__restrict__ w2,
                            __bf16 *__restrict__ w3, __bf16 *__restrict__ w2t, __bf16 *__restrict__ w3t) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < HID * KIN) w1[t] = static_cast<__bf16>(p[OW1 + t]);
  if (t < HID * HID) {
    const int r = t / HID, c = t % HID;
    w2[t] = static_cast<__bf16>(p[OW2 + t]);
    w2t[c * HID + r] = static_cast<__bf16>(p[OW2 + t]);
  }
  if (t < NOUT * HID) {
    const int r = t / HID, c = t % HID;
    w3[t] = static_cast<__bf16>(p[OW3 + t]);
    w3t[c * 32 + r] = static_cast<__bf16>(p[OW3 + t]);   // columns 16..31 stay 0
  }
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                            float *__restrict__ m2, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float a = b1 * m1[t] + (1.0f - b1) * gt;
  const float v = b2 * m2[t] + (1.0f - b2) * gt * gt;
  m1[t] = a;
  m2[t] = v;
  p[t] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Per member: 1 if any correction value of that member is not finite.
__global__ void check_kernel(const float *__restrict__ Y, int ys, int64_t Na, int E, int *__restrict__ bad) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= Na * E) return;
  const int e = static_cast<int>(s % E);
  for (int c = 0; c < 4; ++c)
    if (!isfinite(Y[s * ys + c])) {
      atomicOr(bad + e, 1);
      return;
    }
}

// y_active += dt * Y * out_scale, except for members flagged non-finite.
__global__ void apply_kernel(float *__restrict__ y, const float *__restrict__ Y, int ys, int64_t Na, int E,
                             const int *__restrict__ bad, float4 out_scale, float dt) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= Na * E) return;
  const int e = static_cast<int>(s % E);
  if (bad[e]) return;
  float *o = y + s * 4;
  const float *q = Y + s * ys;
  o[0] += dt * q[0] * out_scale.x;
  o[1] += dt * q[1] * out_scale.y;
  o[2] += dt * q[2] * out_scale.z;
  o[3] += dt * q[3] * out_scale.w;
}

__global__ void scale_out_kernel(const float *__restrict__ Y, int ys, int64_t S, float4 sc, float *__restrict__ out) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= S) return;
  out[s * 4 + 0] = Y[s * ys + 0] * sc.x;
  out[s * 4 + 1] = Y[s * ys + 1] * sc.y;
  out[s * 4 + 2] = Y[s * ys + 2] * sc.z;
  out[s * 4 + 3] = Y[s * ys + 3] * sc.w;
}

__global__ void f64_to_f32_kernel(const double *__restrict__ a, int64_t n, float *__restrict__ b) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) b[t] = static_cast<float>(a[t]);
}

}  // namespace

struct rbffd_closure {
  rbffd_model *model = nullptr;
  int64_t max_s = 0, sp_max = 0;
  float4 inv_in{}, out_sc{};
  DevBuf params, grad, m1, m2, nodef, idx;
  DevBuf w1, w2, w3, w2t, w3t;                       // BF16 weights
  DevBuf X, H1, H2, Y, dY, dY32, dH1, dH2;           // activations [S][.]
  DevBuf XT, H1T, H2T, dH1T, dH2T, dYT;              // transposed [.][Sp]
  DevBuf frag, Yc;                                   // fused forward: packed weights, Y [S][4]
  DevBuf loss, bad;
  int64_t step = 0;
  int act = RBFFD_ACT_TANH;
  int shape = 0;  // fused forward launch shape (rbffd_closure_tune)
};

namespace {

template <int EPI, int NT>
void gemm(hipStream_t s, const __bf16 *A, int lda, const __bf16 *B, int ldb, int M, int K, int k_chunk,
          const float *bias, const __bf16 *H, int ldh, void *C, int ldc, int act = RBFFD_ACT_TANH) {
  dim3 grid((M + 63) / 64, (K + k_chunk - 1) / k_chunk);
  gemm_nt_kernel<EPI, NT><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, K, k_chunk, bias, H, ldh, C, ldc, act);
}

template <class T> const T *cp(const DevBuf &b) { return b.as<T>(); }

// Forward pass for S = Na * E samples of `state` into Y (normalised output).
int forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int64_t S) {
  hipStream_t s = ctx->stream;
  rbffd_model *m = cl->model;
  features_kernel<<<grid_for(S * 40, 256), 256, 0, s>>>(static_cast<const float *>(state), cl->idx.as<int>(), m->Na,
                                                         m->n, m->E, cl->nodef.as<float>(), cl->inv_in,
                                                         cl->X.as<__bf16>());
  const float *p = cl->params.as<float>();
  const int Si = static_cast<int>(S);
  gemm<EPI_ACT, 8>(s, cp<__bf16>(cl->X), KIN, cp<__bf16>(cl->w1), KIN, Si, KIN, KIN, p + OB1, nullptr, 0,
                   cl->H1.p, HID, cl->act);
  gemm<EPI_ACT, 8>(s, cp<__bf16>(cl->H1), HID, cp<__bf16>(cl->w2), HID, Si, HID, HID, p + OB2, nullptr, 0,
                   cl->H2.p, HID, cl->act);
  gemm<EPI_BIAS, 1>(s, cp<__bf16>(cl->H2), HID, cp<__bf16>(cl->w3), HID, Si, HID, HID, p + OB3, nullptr, 0,
                    cl->Y.p, NOUT);
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

// Loss and parameter gradient (into cl->grad) for targets T [S][4].
int backward(rbffd_ctx *ctx, rbffd_closure *cl, const float *T, int64_t S) {
  hipStream_t s = ctx->stream;
  const int Si = static_cast<int>(S);
  const int64_t Sp = (S + 31) / 32 * 32;
  float *g = cl->grad.as<float>();
  RBFFD_HIP(ctx, hipMemsetAsync(cl->grad.p, 0, sizeof(float) * NPARAM, s));
  RBFFD_HIP(ctx, hipMemsetAsync(cl->loss.p, 0, sizeof(double), s));
  loss_kernel<<<grid_for(S, 256), 256, 0, s>>>(cl->Y.as<float>(), T, S, cl->dY.as<__bf16>(), cl->dY32.as<float>(),
                                               cl->loss.as<double>());
  // back through the layers: dH2 = (dY W3) a'(h2), dH1 = (dH2 W2) a'(h1)
  gemm<EPI_DACT, 8>(s, cp<__bf16>(cl->dY), 32, cp<__bf16>(cl->w3t), 32, Si, 32, 32, nullptr, cp<__bf16>(cl->H2),
                    HID, cl->dH2.p, HID, cl->act);
  gemm<EPI_DACT, 8>(s, cp<__bf16>(cl->dH2), HID, cp<__bf16>(cl->w2t), HID, Si, HID, HID, nullptr,
                    cp<__bf16>(cl->H1), HID, cl->dH1.p, HID, cl->act);
  // transposes for the weight gradients (contraction over samples)
  auto tr = [&](const __bf16 *in, int ldi, int Cn, DevBuf &out) {
    dim3 grid(static_cast<unsigned>((Sp + 63) / 64), (Cn + 63) / 64);
    transpose_kernel<<<grid, 256, 0, s>>>(in, ldi, S, Cn, out.as<__bf16>(), Sp);
  };
  tr(cp<__bf16>(cl->X), KIN, KIN, cl->XT);
  tr(cp<__bf16>(cl->H1), HID, HID, cl->H1T);
  tr(cp<__bf16>(cl->H2), HID, HID, cl->H2T);
  tr(cp<__bf16>(cl->dH1), HID, HID, cl->dH1T);
  tr(cp<__bf16>(cl->dH2), HID, HID, cl->dH2T);
  tr(cp<__bf16>(cl->dY), 32, NOUT, cl->dYT);
  const int Ki = static_cast<int>(Sp);
  const int chunk = 1024;
  gemm<EPI_ATOMIC, 10>(s, cp<__bf16>(cl->dH1T), Ki, cp<__bf16>(cl->XT), Ki, HID, Ki, chunk, nullptr, nullptr, 0,
                       g + OW1, KIN);
  gemm<EPI_ATOMIC, 8>(s, cp<__bf16>(cl->dH2T), Ki, cp<__bf16>(cl->H1T), Ki, HID, Ki, chunk, nullptr, nullptr, 0,
                      g + OW2, HID);
  gemm<EPI_ATOMIC, 8>(s, cp<__bf16>(cl->dYT), Ki, cp<__bf16>(cl->H2T), Ki, NOUT, Ki, chunk, nullptr, nullptr, 0,
                      g + OW3, HID);
  const int64_t cch = 2048;
  const unsigned nb = static_cast<unsigned>((S + cch - 1) / cch);
  colsum_kernel<__bf16><<<nb, 128 * COLSUM_SLICES, 0, s>>>(cp<__bf16>(cl->dH1), HID, S, HID, cch, g + OB1);
  colsum_kernel<__bf16><<<nb, 128 * COLSUM_SLICES, 0, s>>>(cp<__bf16>(cl->dH2), HID, S, HID, cch, g + OB2);
  colsum_kernel<float><<<nb, 128 * COLSUM_SLICES, 0, s>>>(cp<float>(cl->dY32), 4, S, 4, cch, g + OB3);
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

void repack(rbffd_closure *cl, hipStream_t s) {
  pack_kernel<<<grid_for(HID * KIN, 256), 256, 0, s>>>(cl->params.as<float>(), cl->w1.as<__bf16>(), cl->w2.as<__bf16>(),
                                                        cl->w3.as<__bf16>(), cl->w2t.as<__bf16>(), cl->w3t.as<__bf16>());
  frag_pack_kernel<<<grid_for(NFRAG * 512, 256), 256, 0, s>>>(cl->params.as<float>(), cl->frag.as<__bf16>());
}

struct MlpShape {
  int T, waves, occ;
};
constexpr MlpShape kMlpShapes[] = {{1, 16, 4}, {1, 8, 4}, {1, 4, 4}, {2, 8, 2}, {2, 4, 2}};
constexpr int kNumMlpShapes = sizeof(kMlpShapes) / sizeof(kMlpShapes[0]);

template <int S, int ACT> auto mlp_kernel() {
  return mlp_forward_kernel<kMlpShapes[S].T, kMlpShapes[S].waves, kMlpShapes[S].occ, ACT>;
}

template <int S> void set_mlp_lds_shape(bool &ok) {
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void *>(mlp_kernel<S, RBFFD_ACT_RELU>()),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(MLP_LDS)) == hipSuccess;
  ok = ok && hipFuncSetAttribute(reinterpret_cast<const void *>(mlp_kernel<S, RBFFD_ACT_TANH>()),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(MLP_LDS)) == hipSuccess;
}

void set_mlp_lds(bool &ok) {
  set_mlp_lds_shape<0>(ok);
  set_mlp_lds_shape<1>(ok);
  set_mlp_lds_shape<2>(ok);
  set_mlp_lds_shape<3>(ok);
  set_mlp_lds_shape<4>(ok);
}

// Fused forward pass into cl->Yc [S][4] in launch shape S. Resident blocks per
// compute unit: as many as LDS (160 KB, 77 KB of packed weights each) and the
// SIMDs' wavefront slots allow; the grid is one wave of them.
template <int SH>
void launch_forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int64_t S) {
  constexpr MlpShape sh = kMlpShapes[SH];
  rbffd_model *m = cl->model;
  constexpr int per_cu = std::min<int>(static_cast<int>((160 * 1024) / MLP_LDS), 4 * sh.occ / sh.waves);
  static_assert(per_cu >= 1, "fused forward launch shape");
  const int64_t units = (S + 16 * sh.T - 1) / (16 * sh.T);
  const unsigned nb = static_cast<unsigned>(
      std::max<int64_t>(1, std::min<int64_t>(static_cast<int64_t>(ctx->n_cu) * per_cu, (units + sh.waves - 1) / sh.waves)));
  auto kern = cl->act == RBFFD_ACT_RELU ? mlp_kernel<SH, RBFFD_ACT_RELU>() : mlp_kernel<SH, RBFFD_ACT_TANH>();
  kern<<<nb, 64 * sh.waves, MLP_LDS, ctx->stream>>>(static_cast<const float *>(state), cl->idx.as<int>(), m->Na, m->n,
                                                    m->E, cl->nodef.as<float>(), cl->inv_in, cl->frag.as<__bf16>(),
                                                    cl->params.as<float>(), cl->Yc.as<float>(), S);
}

int forward_fused(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int64_t S) {
  switch (cl->shape) {
    case 1: launch_forward<1>(ctx, cl, state, S); break;
    case 2: launch_forward<2>(ctx, cl, state, S); break;
    case 3: launch_forward<3>(ctx, cl, state, S); break;
    case 4: launch_forward<4>(ctx, cl, state, S); break;
    default: launch_forward<0>(ctx, cl, state, S); break;
  }
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

}  // namespace

int closure_create(rbffd_ctx *ctx, rbffd_model *m, const rbffd_closure_desc *d, rbffd_closure **out) {
  if (m->physics != RBFFD_PHYS_NS || m->fdt != RBFFD_F32)
    return rbffd_fail(ctx, RBFFD_EINVAL, "the closure needs a Navier-Stokes model with FP32 fields");
  if (m->n > NSLOT_MAX) return rbffd_fail(ctx, RBFFD_EINVAL, "the closure takes stencils of at most 37 nodes");
  if (!d->init_params || !d->node_feature) return rbffd_fail(ctx, RBFFD_EINVAL, "null closure input");
  if (d->activation != RBFFD_ACT_TANH && d->activation != RBFFD_ACT_RELU)
    return rbffd_fail(ctx, RBFFD_EINVAL, "activation must be RBFFD_ACT_TANH or RBFFD_ACT_RELU");
  const int64_t S = m->Na * m->E;
  if (d->max_samples < S || d->max_samples > (int64_t(1) << 28))
    return rbffd_fail(ctx, RBFFD_EINVAL, "max_samples must cover n_active * E (%lld)", (long long)S);
  for (int c = 0; c < 4; ++c)
    if (!(d->in_scale[c] > 0.0f) || !(d->out_scale[c] > 0.0f))
      return rbffd_fail(ctx, RBFFD_EINVAL, "scales must be positive");
  auto *cl = new (std::nothrow) rbffd_closure();
  if (!cl) return rbffd_fail(ctx, RBFFD_ENOMEM, "host allocation");
  cl->model = m;
  cl->act = d->activation;
  cl->max_s = d->max_samples;
  cl->sp_max = (d->max_samples + 31) / 32 * 32;
  cl->inv_in = make_float4(1.0f / d->in_scale[0], 1.0f / d->in_scale[1], 1.0f / d->in_scale[2], 1.0f / d->in_scale[3]);
  cl->out_sc = make_float4(d->out_scale[0], d->out_scale[1], d->out_scale[2], d->out_scale[3]);
  const size_t Sx = static_cast<size_t>(cl->max_s), Sp = static_cast<size_t>(cl->sp_max), b2 = 2;
  bool ok = cl->params.alloc(4 * NPARAM) == hipSuccess && cl->grad.alloc(4 * NPARAM) == hipSuccess &&
            cl->m1.alloc(4 * NPARAM) == hipSuccess && cl->m2.alloc(4 * NPARAM) == hipSuccess &&
            cl->nodef.alloc(4 * m->Na) == hipSuccess && cl->idx.alloc(4 * m->Na * m->n) == hipSuccess &&
            cl->w1.alloc(b2 * HID * KIN) == hipSuccess && cl->w2.alloc(b2 * HID * HID) == hipSuccess &&
            cl->w3.alloc(b2 * NOUT * HID) == hipSuccess && cl->w2t.alloc(b2 * HID * HID) == hipSuccess &&
            cl->w3t.alloc(b2 * HID * 32) == hipSuccess && cl->X.alloc(b2 * Sx * KIN) == hipSuccess &&
            cl->H1.alloc(b2 * Sx * HID) == hipSuccess && cl->H2.alloc(b2 * Sx * HID) == hipSuccess &&
            cl->Y.alloc(4 * Sx * NOUT) == hipSuccess && cl->dY.alloc(b2 * Sx * 32) == hipSuccess &&
            cl->dY32.alloc(4 * Sx * 4) == hipSuccess && cl->dH1.alloc(b2 * Sx * HID) == hipSuccess &&
            cl->dH2.alloc(b2 * Sx * HID) == hipSuccess && cl->XT.alloc(b2 * KIN * Sp) == hipSuccess &&
            cl->H1T.alloc(b2 * HID * Sp) == hipSuccess && cl->H2T.alloc(b2 * HID * Sp) == hipSuccess &&
            cl->dH1T.alloc(b2 * HID * Sp) == hipSuccess && cl->dH2T.alloc(b2 * HID * Sp) == hipSuccess &&
            cl->dYT.alloc(b2 * NOUT * Sp) == hipSuccess && cl->loss.alloc(8) == hipSuccess &&
            cl->bad.alloc(4 * m->E) == hipSuccess && cl->frag.alloc(b2 * NFRAG * 512) == hipSuccess &&
            cl->Yc.alloc(4 * Sx * 4) == hipSuccess;
  if (!ok) {
    delete cl;
    return rbffd_fail(ctx, RBFFD_ENOMEM, "device allocation (closure)");
  }
  bool lds_ok = true;
  set_mlp_lds(lds_ok);
  if (!lds_ok) {
    delete cl;
    return rbffd_fail(ctx, RBFFD_EDEVICE, "closure: LDS size of the fused forward kernel");
  }
  hipStream_t s = ctx->stream;
  bool cp_ok = hipMemcpyAsync(cl->params.p, d->init_params, 4 * NPARAM, hipMemcpyDeviceToDevice, s) == hipSuccess &&
               hipMemsetAsync(cl->m1.p, 0, 4 * NPARAM, s) == hipSuccess &&
               hipMemsetAsync(cl->m2.p, 0, 4 * NPARAM, s) == hipSuccess &&
               hipMemsetAsync(cl->w3t.p, 0, b2 * HID * 32, s) == hipSuccess &&
               hipMemsetAsync(cl->w3.p, 0, b2 * NOUT * HID, s) == hipSuccess;
  if (!cp_ok) {
    delete cl;
    return rbffd_fail(ctx, RBFFD_EDEVICE, "closure set-up copies");
  }
  f64_to_f32_kernel<<<grid_for(m->Na, 256), 256, 0, s>>>(d->node_feature, m->Na, cl->nodef.as<float>());
  const int64_t cnt = m->Na * m->n;
  const hipError_t e_idx = hipMemcpyAsync(cl->idx.p, m->idx_t.p, sizeof(int) * cnt, hipMemcpyDeviceToDevice, s);
  repack(cl, s);
  const hipError_t e_launch = hipGetLastError();
  const hipError_t e_sync = hipStreamSynchronize(s);
  if (e_idx != hipSuccess || e_launch != hipSuccess || e_sync != hipSuccess) {
    delete cl;
    return rbffd_fail(ctx, RBFFD_EDEVICE, "closure set-up: index copy %s, launches %s, synchronisation %s",
                      hipGetErrorString(e_idx), hipGetErrorString(e_launch), hipGetErrorString(e_sync));
  }
  *out = cl;
  return RBFFD_OK;
}

int closure_destroy(rbffd_closure *cl) {
  delete cl;
  return RBFFD_OK;
}

float *closure_params(rbffd_closure *cl) { return cl->params.as<float>(); }

int closure_forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, float *out) {
  const int64_t S = cl->model->Na * cl->model->E;
  int rc = forward_fused(ctx, cl, state, S);
  if (rc) return rc;
  scale_out_kernel<<<grid_for(S, 256), 256, 0, ctx->stream>>>(cl->Yc.as<float>(), 4, S, cl->out_sc, out);
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

// Time every launch shape of the fused forward kernel on `state` (one
// untimed call, then three timed ones each) and keep the fastest; with
// *chosen >= 0 on entry, time and keep that shape only.
int closure_tune(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int *chosen, double *best_us) {
  const int64_t S = cl->model->Na * cl->model->E;
  if (*chosen >= kNumMlpShapes) return rbffd_fail(ctx, RBFFD_EINVAL, "closure shape %d outside -1..%d", *chosen,
                                                  kNumMlpShapes - 1);
  const int first = *chosen >= 0 ? *chosen : 0, last = *chosen >= 0 ? *chosen : kNumMlpShapes - 1;
  hipEvent_t e0, e1;
  RBFFD_HIP(ctx, hipEventCreate(&e0));
  RBFFD_HIP(ctx, hipEventCreate(&e1));
  int best = first;
  double best_t = -1.0;
  int rc = RBFFD_OK;
  for (int sh = first; sh <= last && rc == RBFFD_OK; ++sh) {
    cl->shape = sh;
    rc = forward_fused(ctx, cl, state, S);
    if (rc) break;
    if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = RBFFD_EDEVICE;
    for (int r = 0; r < 3 && rc == RBFFD_OK; ++r) rc = forward_fused(ctx, cl, state, S);
    float ms = 0.0f;
    if (rc == RBFFD_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = rbffd_fail(ctx, RBFFD_EDEVICE, "closure tuning: event timing");
    const double us = 1e3 * ms / 3.0;
    if (rc == RBFFD_OK && (best_t < 0.0 || us < best_t)) {
      best_t = us;
      best = sh;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cl->shape = best;
  if (rc) return rc;
  *chosen = best;
  *best_us = best_t;
  return RBFFD_OK;
}

int closure_gradient(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, float *grad,
                     double *loss) {
  const int64_t S = cl->model->Na * cl->model->E;
  int rc = forward(ctx, cl, state, S);
  if (!rc) rc = backward(ctx, cl, target, S);
  if (rc) return rc;
  if (grad) RBFFD_HIP(ctx, hipMemcpyAsync(grad, cl->grad.p, 4 * NPARAM, hipMemcpyDeviceToDevice, ctx->stream));
  RBFFD_HIP(ctx, hipMemcpyAsync(loss, cl->loss.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  RBFFD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return RBFFD_OK;
}

int closure_train_step(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, double lr,
                       double *loss) {
  int rc = closure_gradient(ctx, cl, state, target, nullptr, loss);
  if (rc) return rc;
  cl->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, static_cast<float>(cl->step)), c2 = 1.0f - powf(b2, static_cast<float>(cl->step));
  adam_kernel<<<grid_for(NPARAM, 256), 256, 0, ctx->stream>>>(cl->params.as<float>(), cl->grad.as<float>(),
                                                              cl->m1.as<float>(), cl->m2.as<float>(), NPARAM,
                                                              static_cast<float>(lr), b1, b2, 1e-8f, c1, c2);
  repack(cl, ctx->stream);
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

int closure_step(rbffd_ctx *ctx, rbffd_closure *cl, void *state, double *t, double dt, int64_t n_steps, int tableau,
                 int64_t *n_fallback) {
  rbffd_model *m = cl->model;
  const int64_t S = m->Na * m->E;
  hipStream_t s = ctx->stream;
  int64_t fb = 0;
  std::vector<int> hb(m->E);
  for (int64_t k = 0; k < n_steps; ++k) {
    int rc = model_ghost(ctx, m, state);
    if (!rc) rc = forward_fused(ctx, cl, state, S);  // correction of the state before the step
    if (!rc) rc = model_step(ctx, m, state, t, dt, 1, tableau);
    if (rc) return rc;
    RBFFD_HIP(ctx, hipMemsetAsync(cl->bad.p, 0, sizeof(int) * m->E, s));
    check_kernel<<<grid_for(S, 256), 256, 0, s>>>(cl->Yc.as<float>(), 4, m->Na, m->E, cl->bad.as<int>());
    apply_kernel<<<grid_for(S, 256), 256, 0, s>>>(static_cast<float *>(state), cl->Yc.as<float>(), 4, m->Na, m->E,
                                                  cl->bad.as<int>(), cl->out_sc, static_cast<float>(dt));
    RBFFD_HIP(ctx, hipGetLastError());
    if (n_fallback) {
      RBFFD_HIP(ctx, hipMemcpyAsync(hb.data(), cl->bad.p, sizeof(int) * m->E, hipMemcpyDeviceToHost, s));
      RBFFD_HIP(ctx, hipStreamSynchronize(s));
      for (int v : hb) fb += v;
    }
  }
  if (n_fallback) *n_fallback = fb;
  return RBFFD_OK;
}

// Launch the matrix-core probe: four 256-thread blocks per compute unit.
int mfma_probe(rbffd_ctx *ctx, int shape, float *out, int64_t n_out, int iters, int64_t *flops) {
  const int64_t blocks = 4 * static_cast<int64_t>(ctx->n_cu);
  if (!out || iters < 1 || (shape != 0 && shape != 1) || n_out < blocks * 256)
    return rbffd_fail(ctx, RBFFD_EINVAL, "mfma probe: needs shape 0 or 1, iters >= 1 and %lld output floats",
                      static_cast<long long>(blocks * 256));
  if (shape == 0)
    mfma_probe_kernel<0><<<static_cast<unsigned>(blocks), 256, 0, ctx->stream>>>(out, iters);
  else
    mfma_probe_kernel<1><<<static_cast<unsigned>(blocks), 256, 0, ctx->stream>>>(out, iters);
  RBFFD_HIP(ctx, hipGetLastError());
  // 4 wavefronts per block, 4 products per round of 16 x 16 x 32 or 32 x 32 x 16 multiply-adds
  const int64_t per = shape == 0 ? 2 * 16 * 16 * 32 : 2 * 32 * 32 * 16;
  *flops = blocks * 4 * static_cast<int64_t>(iters) * 4 * per;
  return RBFFD_OK;
}
