// Learned surrogate of the per-neighbourhood conditional density: a small
// MLP maps a neighbourhood's range-scaled geometry (the m neighbours'
// offsets from the observation, divided by the range, in NNarray column
// order), the smoothness and the nugget ratio to the kriging weights b and
// the log conditional variance log(v / sigma2) of Eq. (3).  The network
// runs in BF16 on the matrix cores (v_mfma_f32_32x32x16_bf16, FP32
// accumulation); the log-likelihood terms it feeds are formed in FP64.
//
// Network: 64 inputs (2m = 60 offsets, nu, tau2, two zero pads) -> 256 ->
// 256 -> 256 -> 32 outputs (m weights, log variance, one pad), SiLU after
// each hidden layer.  Parameters, in this order, row-major W[out][in]:
//   W0[256][64] b0[256] W1[256][256] b1[256] W2[256][256] b2[256]
//   W3[32][256] b3[32]
// kept as an FP32 master copy (optimiser) and a BF16 copy (compute).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "vecchia.h"
#include "vecchia_surrogate.h"

namespace vecchia_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kIn = VEC_MLP_IN, kHid = VEC_MLP_HIDDEN, kOut = VEC_MLP_OUT;
constexpr int kM = VEC_SURROGATE_M;
static_assert(2 * kM + 2 <= kIn && kM + 1 <= kOut, "network dimensions");

// element offsets of the parameter blocks
constexpr int64_t kOffW[4] = {0, kHid * kIn + kHid, kHid * kIn + kHid + kHid * kHid + kHid,
                              kHid * kIn + kHid + 2 * (kHid * kHid + kHid)};
constexpr int64_t kOffB[4] = {kOffW[0] + kHid * kIn, kOffW[1] + kHid * kHid,
                              kOffW[2] + kHid * kHid, kOffW[3] + kOut * kHid};
constexpr int64_t kParams = kOffB[3] + kOut;
constexpr int kLayerIn[4] = {kIn, kHid, kHid, kHid};
constexpr int kLayerOut[4] = {kHid, kHid, kHid, kOut};

// logistic function with the hardware reciprocal (about 1 ulp; the result is
// rounded to BF16 or feeds an FP32 gradient, so a correctly rounded divide
// would change nothing that is kept); z -> -inf gives 1/inf = 0
__device__ __forceinline__ float sigmoidf(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// ---------------------------------------------------------------------------
// C[M][N] = op(A)[M][K] * op(B)[K][N] on the matrix cores, one wave per 32x32
// tile.  op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k];
// op(B)(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n].  M, N multiples of 32,
// the K range [k_begin, k_end) a multiple of 16 (the host checks).
// Accumulator lane layout of the 32x32x16 instruction: lane l holds column
// l % 32 and rows 8 (j / 4) + 4 (l / 32) + j % 4 for j = 0..15; operand
// lanes hold row (A) / column (B) l % 32 and k = 8 (l / 32) + 0..7.
// ---------------------------------------------------------------------------
enum Epi { kEpiHidden = 0, kEpiOut = 1, kEpiBackAct = 2, kEpiAtomic = 3 };

struct GemmArgs {
  int M, N, k_begin, k_end, k_split;
  const __bf16* A;
  int lda;
  const __bf16* B;
  int ldb;
  const float* bias;  // kEpiHidden, kEpiOut: [N]
  float* Z;           // kEpiHidden: pre-activation out (nullable); kEpiBackAct: pre-activation in
  int ldz;
  __bf16* H;  // kEpiHidden: activation out; kEpiBackAct: gradient out
  int ldh;
  float* C;  // kEpiOut: output; kEpiAtomic: accumulated
  int ldc;
};

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(64) void gemm_kernel(const GemmArgs g) {
  const int l = threadIdx.x;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int lr = l & 31, kh = 8 * (l >> 5);
  int kb = g.k_begin, ke = g.k_end;
  if (g.k_split > 0) {  // split-K: this z-slice's share of the range
    kb = g.k_begin + blockIdx.z * g.k_split;
    ke = min(kb + g.k_split, g.k_end);
  }
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x8 a, b;
    if constexpr (!TA) {
      a = *reinterpret_cast<const bf16x8*>(g.A + (int64_t)(m0 + lr) * g.lda + k0 + kh);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = g.A[(int64_t)(k0 + kh + j) * g.lda + m0 + lr];
    }
    if constexpr (TB) {
      b = *reinterpret_cast<const bf16x8*>(g.B + (int64_t)(n0 + lr) * g.ldb + k0 + kh);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = g.B[(int64_t)(k0 + kh + j) * g.ldb + n0 + lr];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int c = n0 + lr;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int r = m0 + 8 * (j >> 2) + 4 * (l >> 5) + (j & 3);
    const float v = acc[j];
    if constexpr (EPI == kEpiHidden) {
      const float z = v + g.bias[c];
      if (g.Z) g.Z[(int64_t)r * g.ldz + c] = z;
      g.H[(int64_t)r * g.ldh + c] = (__bf16)(z * sigmoidf(z));
    } else if constexpr (EPI == kEpiOut) {
      g.C[(int64_t)r * g.ldc + c] = v + g.bias[c];
    } else if constexpr (EPI == kEpiBackAct) {
      const float z = g.Z[(int64_t)r * g.ldz + c];
      const float s = sigmoidf(z);
      g.H[(int64_t)r * g.ldh + c] = (__bf16)(v * s * (1.0f + z * (1.0f - s)));
    } else {
      atomicAdd(&g.C[(int64_t)r * g.ldc + c], v);
    }
  }
}

template <bool TA, bool TB, int EPI>
static hipError_t gemm(const GemmArgs& g, int kz, hipStream_t st) {
  hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI>), dim3(g.N / 32, g.M / 32, kz), dim3(64), 0, st,
                     g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inference: the whole network in one launch, one wave per 32 rows, the
// activations never leaving registers.  Each layer is computed transposed,
// out^T (features x rows) = W (features x in) * in^T, so the weights are the
// A operand (lane = output feature) and the activations the B operand
// (lane = row).  The accumulator of output tile t then holds, in lane l, row
// l % 32 and features 32 t + 8 (j / 4) + 4 (l / 32) + j % 4 (j = 0..15); its
// halves j = 0..7 and 8..15, rounded to BF16 after bias and SiLU, are exactly
// a B operand of the next layer (lane l % 32 = row, k = 8 (l / 32) + i) if
// that layer's A operand takes input features in the same order: k = 8 g + i
// of step s = (t, h) is input feature 32 t + 16 h + 8 (i / 4) + 4 g + i % 4.
// The BF16 rounding points are those of the layer-by-layer path (hidden
// activations rounded, FP32 accumulation).
//
// The weights are first copied into fragment order: fragment f of a layer is
// 64 lanes x 8 BF16, lane l's eight A-operand values contiguous, so each
// MFMA operand is one coalesced 1 KiB load.  Fragments per layer: layer 0,
// f = 4 t' + c (output tile t', input chunk c of 16 natural-order inputs);
// layers 1, 2, f = 16 t' + s; layer 3, f = s.
// ---------------------------------------------------------------------------
constexpr int64_t kFragOff[4] = {0, kHid * kIn, kHid * kIn + kHid * kHid,
                                 kHid * kIn + 2 * kHid * kHid};
constexpr int64_t kFragElems = kFragOff[3] + kOut * kHid;

__global__ __launch_bounds__(256) void pack_fragments_kernel(const __bf16* __restrict__ Pb,
                                                             __bf16* __restrict__ F) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= kFragElems) return;
  const int L = e < kFragOff[1] ? 0 : (e < kFragOff[2] ? 1 : (e < kFragOff[3] ? 2 : 3));
  const int64_t r = e - kFragOff[L];
  const int i = (int)(r & 7), l = (int)((r >> 3) & 63), f = (int)(r >> 9);
  const int lr = l & 31, g = l >> 5;
  int64_t src;
  if (L == 0) {
    src = (int64_t)(32 * (f >> 2) + lr) * kIn + 16 * (f & 3) + 8 * g + i;
  } else {
    const int tp = (L == 3) ? 0 : (f >> 4), st = f & 15;
    src = (int64_t)(32 * tp + lr) * kHid + 16 * st + 8 * (i >> 2) + 4 * g + (i & 3);
  }
  F[e] = Pb[kOffW[L] + src];
}

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// bias + SiLU of four output tiles 4 tq .. 4 tq + 3 into act[tile][half]
__device__ __forceinline__ void hidden_epilogue(const f32x16 (&acc)[4], int tq, int g,
                                                const float* __restrict__ bias,
                                                bf16x8 (&act)[8][2]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = 4 * tq + u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = *reinterpret_cast<const float4*>(bias + 32 * t + 8 * q + 4 * g);
      const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * q + e;
        const float z = acc[u][j] + bb[e];
        act[t][j >> 3][j & 7] = (__bf16)(z * sigmoidf(z));
      }
    }
  }
}

// NS steps of four MFMAs into acc[0..3]: step s multiplies fragment
// frag(u, s) by B operand bop(u, s) (u = 0..3); the fragments of step
// s + kAhead are loaded while step s multiplies.
template <int NS, typename FragPtr, typename BOp>
__device__ __forceinline__ void mfma_steps4(f32x16 (&acc)[4], FragPtr frag, BOp bop) {
  constexpr int kAhead = 3;
  bf16x8 fr[kAhead + 1][4];
#pragma unroll
  for (int s = 0; s < kAhead && s < NS; ++s) {
#pragma unroll
    for (int u = 0; u < 4; ++u) fr[s][u] = load8(frag(u, s));
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s + kAhead < NS) {
#pragma unroll
      for (int u = 0; u < 4; ++u) fr[(s + kAhead) % (kAhead + 1)][u] = load8(frag(u, s + kAhead));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fr[s % (kAhead + 1)][u], bop(u, s),
                                                       acc[u], 0, 0, 0);
  }
}

__global__ __launch_bounds__(256, 2) void mlp_infer_kernel(int64_t rows, const __bf16* __restrict__ x,
                                                        const float* __restrict__ P,
                                                        const __bf16* __restrict__ F,
                                                        float* __restrict__ y) {
  static_assert(kIn == 64 && kHid == 256 && kOut == 32, "fused inference layout");
  const int l = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
  if (r0 >= rows) return;  // rows is a multiple of 32: a wave has all or none
  const int lr = l & 31, g = l >> 5;
  const __bf16* Fl = F + 8 * l;  // this lane's eight values of every fragment
  bf16x8 act[8][2];
  {  // layer 0: 64 inputs in natural order, chunks c of 16
    bf16x8 xin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) xin[c] = load8(x + (r0 + lr) * kIn + 16 * c + 8 * g);
#pragma unroll
    for (int tq = 0; tq < 2; ++tq) {
      f32x16 acc[4] = {};
      mfma_steps4<4>(
          acc, [&](int u, int c) { return Fl + kFragOff[0] + 512 * (4 * (4 * tq + u) + c); },
          [&](int, int c) { return xin[c]; });
      hidden_epilogue(acc, tq, g, P + kOffB[0], act);
    }
  }
#pragma unroll
  for (int L = 1; L < 3; ++L) {  // hidden layers 1 and 2
    bf16x8 nxt[8][2];
#pragma unroll
    for (int tq = 0; tq < 2; ++tq) {
      f32x16 acc[4] = {};
      mfma_steps4<16>(
          acc, [&](int u, int s) { return Fl + kFragOff[L] + 512 * (16 * (4 * tq + u) + s); },
          [&](int, int s) { return act[s >> 1][s & 1]; });
      hidden_epilogue(acc, tq, g, P + kOffB[L], nxt);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      act[t][0] = nxt[t][0];
      act[t][1] = nxt[t][1];
    }
  }
  // output layer: one tile of 32 outputs, four partial accumulators over
  // the steps (s = 4 v + u) summed at the end
  f32x16 acc[4] = {};
  mfma_steps4<4>(
      acc, [&](int u, int v) { return Fl + kFragOff[3] + 512 * (4 * v + u); },
      [&](int u, int v) { return act[(4 * v + u) >> 1][(4 * v + u) & 1]; });
  float* yr = y + (r0 + lr) * kOut;
  const float* b3 = P + kOffB[3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = 8 * q + 4 * g;
    const float4 b = *reinterpret_cast<const float4*>(b3 + o);
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * q + e;
      v[e] = (acc[0][j] + acc[1][j]) + (acc[2][j] + acc[3][j]);
    }
    *reinterpret_cast<float4*>(yr + o) =
        make_float4(v[0] + b.x, v[1] + b.y, v[2] + b.z, v[3] + b.w);
  }
}

// loss = sum_r sum_c w_c (Y - T)^2 * scale;  dY = 2 w_c (Y - T) scale (BF16)
__global__ __launch_bounds__(256) void loss_kernel(int rows, const float* __restrict__ Y,
                                                   const float* __restrict__ T,
                                                   const float* __restrict__ colw, float scale,
                                                   __bf16* __restrict__ dY,
                                                   double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t total = (int64_t)rows * kOut;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int c = (int)(e % kOut);
    const float d = Y[e] - T[e];
    const float w = colw[c];
    s += (double)(w * d * d) * scale;
    dY[e] = (__bf16)(2.0f * w * d * scale);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// db[c] += sum_r dZ[r][c]: one workgroup per 32 columns, 32 row phases;
// phase q sums rows q, q + 32, ... in order, then the phases are added in a
// fixed tree, so the result does not depend on timing
__global__ __launch_bounds__(1024) void colsum_kernel(int rows, int cols,
                                                      const __bf16* __restrict__ dZ,
                                                      float* __restrict__ db) {
  __shared__ float part[32][33];
  const int cl = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cl;
  float s = 0.0f;
  if (c < cols) {
    for (int r = q; r < rows; r += 32) s += (float)dZ[(int64_t)r * cols + c];
  }
  part[q][cl] = s;
  __syncthreads();
  for (int w = 16; w > 0; w >>= 1) {
    if (q < w) part[q][cl] += part[q + w][cl];
    __syncthreads();
  }
  if (q == 0 && c < cols) db[c] += part[0][cl];
}

__global__ void zero_f32_kernel(float* __restrict__ x, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

__global__ void adam_kernel(int64_t count, float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2,
                            __bf16* __restrict__ wb, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float a = b1 * m1[e] + (1.0f - b1) * gi;
    const float b = b2 * m2[e] + (1.0f - b2) * gi * gi;
    m1[e] = a;
    m2[e] = b;
    const float x = w[e] - lr * (a * c1) / (sqrtf(b * c2) + eps);
    w[e] = x;
    wb[e] = (__bf16)x;
  }
}

__global__ void to_bf16_kernel(int64_t count, const float* __restrict__ x,
                               __bf16* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (__bf16)x[e];
}

// Inputs of observation i (one thread each): offsets of its m = kM
// neighbours, divided by the range, in NNarray column order; nu; tau2;
// zeros.  flag[i] = 1 marks observations the network does not serve: fewer
// than m neighbours, a malformed row, or a scaled offset outside [dist_lo,
// dist_hi] in length.  The neighbour indices are read first and the
// coordinates after, so all loads of a thread are in flight together; the
// row is written as eight 16-byte stores.
// The offsets are defined as FP32 values rounded to BF16; the empty asm
// keeps the compiler from folding the two conversions into one direct
// FP64 -> BF16 rounding, which differs in rare double-rounding cases.
__device__ __forceinline__ float as_f32(double v) {
  float f = (float)v;
  asm("" : "+v"(f));
  return f;
}

__global__ __launch_bounds__(256) void features_kernel(
    int64_t i0, int64_t count, const double* __restrict__ locs, const int32_t* __restrict__ NN,
    const double* __restrict__ covparms, double nu, float dist_lo, float dist_hi,
    __bf16* __restrict__ feat, uint8_t* __restrict__ flag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int64_t i = i0 + t;
  const double ir = 1.0 / covparms[1];
  const double tau2 = covparms[2];
  const double xi = locs[2 * i], yi = locs[2 * i + 1];
  const int32_t* row = NN + i * (int64_t)(kM + 1);
  bool out = i < kM || row[0] != (int32_t)i;
  int64_t nb[kM];
#pragma unroll
  for (int j = 0; j < kM; ++j) {
    const int64_t v = row[1 + j];
    const bool ok = v >= 0 && v < i;
    out = out || !ok;
    nb[j] = ok ? v : i;  // a stand-in inside the array; the row is flagged anyway
  }
  bf16x8 f[kIn / 8];
#pragma unroll
  for (int j = 0; j < kM; ++j) {
    const float dx = as_f32((locs[2 * nb[j]] - xi) * ir);
    const float dy = as_f32((locs[2 * nb[j] + 1] - yi) * ir);
    const float len = sqrtf(dx * dx + dy * dy);
    out = out || len < dist_lo || len > dist_hi;
    const bool ok = nb[j] != i;
    f[(2 * j) >> 3][(2 * j) & 7] = (__bf16)(ok ? dx : 0.0f);
    f[(2 * j + 1) >> 3][(2 * j + 1) & 7] = (__bf16)(ok ? dy : 0.0f);
  }
  f[(2 * kM) >> 3][(2 * kM) & 7] = (__bf16)as_f32(nu);
  f[(2 * kM + 1) >> 3][(2 * kM + 1) & 7] = (__bf16)as_f32(tau2);
#pragma unroll
  for (int e = 2 * kM + 2; e < kIn; ++e) f[e >> 3][e & 7] = (__bf16)0.0f;
  bf16x8* dst = reinterpret_cast<bf16x8*>(feat + t * kIn);
#pragma unroll
  for (int q = 0; q < kIn / 8; ++q) dst[q] = f[q];
  if (flag) flag[t] = out ? 1 : 0;
}

// FP64 log-likelihood sums (logdet, ySy, XSX, ySX) of the observations the
// network serves, from its outputs Y[t] = (b_1..b_m, scaled log variance):
// e_y = y_i - b.y_s, e_X = X_i - b.X_s, v = sigma2 exp(lv).  An observation
// is handed back (its index appended to `back`) if flagged by the feature
// pass or if lv leaves the range a conditional variance can take,
// [log tau2, log(1 + tau2)] widened by lv_slack, or lies below lv_floor.
template <int PC>
__global__ __launch_bounds__(256) void sums_kernel(
    int64_t i0, int64_t count, const int32_t* __restrict__ NN, const double* __restrict__ y,
    const double* __restrict__ X, const double* __restrict__ covparms,
    const float* __restrict__ Y, const uint8_t* __restrict__ flag, float lv_scale,
    float lv_shift, float lv_slack, float lv_floor, double* __restrict__ partials,
    int32_t* __restrict__ back, unsigned int* __restrict__ nback) {
  constexpr int NR = 2 + PC * PC + PC;
  __shared__ double red[NR][256];
  double acc[NR];
#pragma unroll
  for (int e = 0; e < NR; ++e) acc[e] = 0.0;
  const double sigma2 = covparms[0], tau2 = covparms[2];
  const double lv_lo = fmax(log(tau2) - lv_slack, (double)lv_floor);
  const double lv_hi = log1p(tau2) + lv_slack;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + t;
    // network outputs: 32 floats, eight 16-byte loads
    float yt[kOut];
#pragma unroll
    for (int q = 0; q < kOut / 4; ++q) {
      const float4 v = reinterpret_cast<const float4*>(Y + t * kOut)[q];
      yt[4 * q] = v.x;
      yt[4 * q + 1] = v.y;
      yt[4 * q + 2] = v.z;
      yt[4 * q + 3] = v.w;
    }
    const double lv = (double)yt[kM] * lv_scale + lv_shift;
    const int32_t* row = NN + i * (int64_t)(kM + 1);
    bool give_back = (flag && flag[t]) || !(lv >= lv_lo && lv <= lv_hi) || i < kM;
    int64_t nb[kM];
#pragma unroll
    for (int j = 0; j < kM; ++j) {
      const int64_t v = row[1 + j];
      const bool ok = v >= 0 && v < i;
      give_back = give_back || !ok;
      nb[j] = ok ? v : i;  // a stand-in inside the array; the row is handed back anyway
    }
    if (!give_back) {
      double ey = y[i], eX[PC];
#pragma unroll
      for (int q = 0; q < PC; ++q) eX[q] = X[i * PC + q];
#pragma unroll
      for (int j = 0; j < kM; ++j) {
        const double b = (double)yt[j];
        ey -= b * y[nb[j]];
#pragma unroll
        for (int q = 0; q < PC; ++q) eX[q] -= b * X[nb[j] * PC + q];
      }
      const double v = sigma2 * exp(lv), iv = 1.0 / v;
      acc[0] += log(v);
      acc[1] += ey * ey * iv;
#pragma unroll
      for (int a = 0; a < PC; ++a) {
#pragma unroll
        for (int b = 0; b < PC; ++b) acc[2 + a * PC + b] += eX[a] * eX[b] * iv;
        acc[2 + PC * PC + a] += ey * eX[a] * iv;
      }
    } else {
      back[atomicAdd(nback, 1u)] = (int32_t)i;
    }
  }
#pragma unroll
  for (int e = 0; e < NR; ++e) red[e][threadIdx.x] = acc[e];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int e = 0; e < NR; ++e) red[e][threadIdx.x] += red[e][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < NR) partials[(int64_t)blockIdx.x * NR + threadIdx.x] = red[threadIdx.x][0];
}

// raw[e] (+)= sum_b partials[b][e]: one workgroup per entry, thread t adds
// rows t, t + 256, ... in order, then a fixed tree over the threads
__global__ __launch_bounds__(256) void sum_rows_kernel(const double* __restrict__ partials,
                                                       int rows, int nr, double* __restrict__ raw,
                                                       int accumulate) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < rows; b += 256) s += partials[(int64_t)b * nr + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) raw[e] = accumulate ? raw[e] + red[0] : red[0];
}

}  // namespace vecchia_mlp

using namespace vecchia_mlp;

namespace {

int hip_rc(hipError_t e) { return e == hipSuccess ? VEC_OK : VEC_EHIP; }

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace carve-up for `rows` rows (training adds pre-activations and
// gradient buffers)
struct MlpWork {
  __bf16 *h[3], *dy, *dh[2];
  float *z[3], *y;
  size_t bytes;
};

MlpWork carve(void* ws, int64_t rows, bool training) {
  MlpWork w = {};
  char* p = static_cast<char*>(ws);
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* q = p ? p + o : nullptr;
    o += al256(bytes);
    return q;
  };
  const size_t hb = (size_t)rows * kHid * sizeof(__bf16), zb = (size_t)rows * kHid * sizeof(float);
  for (int L = 0; L < 3; ++L) w.h[L] = reinterpret_cast<__bf16*>(take(hb));
  w.y = reinterpret_cast<float*>(take((size_t)rows * kOut * sizeof(float)));
  if (training) {
    for (int L = 0; L < 3; ++L) w.z[L] = reinterpret_cast<float*>(take(zb));
    w.dy = reinterpret_cast<__bf16*>(take((size_t)rows * kOut * sizeof(__bf16)));
    for (int L = 0; L < 2; ++L) w.dh[L] = reinterpret_cast<__bf16*>(take(hb));
  }
  w.bytes = o;
  return w;
}

bool rows_ok(int64_t rows) { return rows > 0 && rows % 32 == 0 && rows <= (1 << 24); }

// forward pass: hidden layers into w.h[0..2] (pre-activations into w.z when
// training), output into y
int forward(int64_t rows, const __bf16* x, const float* P, const __bf16* Pb, float* y,
            const MlpWork& w, bool training, hipStream_t st) {
  const __bf16* in = x;
  for (int L = 0; L < 4; ++L) {
    GemmArgs g = {};
    g.M = (int)rows;
    g.N = kLayerOut[L];
    g.k_begin = 0;
    g.k_end = kLayerIn[L];
    g.A = in;
    g.lda = kLayerIn[L];
    g.B = Pb + kOffW[L];
    g.ldb = kLayerIn[L];
    g.bias = P + kOffB[L];
    hipError_t e;
    if (L < 3) {
      g.Z = training ? w.z[L] : nullptr;
      g.ldz = kHid;
      g.H = w.h[L];
      g.ldh = kHid;
      e = gemm<false, true, kEpiHidden>(g, 1, st);
      in = w.h[L];
    } else {
      g.C = y;
      g.ldc = kOut;
      e = gemm<false, true, kEpiOut>(g, 1, st);
    }
    if (e != hipSuccess) return VEC_EHIP;
  }
  return VEC_OK;
}

}  // namespace

extern "C" {

int64_t vec_mlp_param_count(void) { return kParams; }

size_t vec_mlp_workspace_bytes(int64_t rows, int32_t training) {
  if (!rows_ok(rows)) return 0;
  if (!training) return al256((size_t)kFragElems * sizeof(__bf16));  // weights in fragment order
  return carve(nullptr, rows, true).bytes;
}

int vec_mlp_forward(int64_t rows, const uint16_t* x, const float* params,
                    const uint16_t* params_bf16, float* y, void* workspace,
                    size_t workspace_bytes, void* stream) {
  auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (!rows_ok(rows) || !x || !params || !params_bf16 || !y || !workspace) return VEC_EINVAL;
  if (!a16(x) || !a16(params) || !a16(y) || !a16(workspace)) return VEC_EINVAL;
  if (workspace_bytes < (size_t)kFragElems * sizeof(__bf16)) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  __bf16* F = static_cast<__bf16*>(workspace);
  hipLaunchKernelGGL(pack_fragments_kernel, dim3((unsigned)((kFragElems + 255) / 256)), dim3(256),
                     0, st, reinterpret_cast<const __bf16*>(params_bf16), F);
  const int64_t blocks = (rows / 32 + 3) / 4;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)blocks), dim3(256), 0, st, rows,
                     reinterpret_cast<const __bf16*>(x), params, F, y);
  return hip_rc(hipGetLastError());
}

int vec_mlp_loss_grad(int64_t rows, const uint16_t* x, const float* targets, const float* colw,
                      float scale, const float* params, const uint16_t* params_bf16, float* grad,
                      double* loss, void* workspace, size_t workspace_bytes, void* stream) {
  if (!rows_ok(rows) || !x || !targets || !colw || !params || !params_bf16 || !grad || !loss ||
      !workspace)
    return VEC_EINVAL;
  const MlpWork w = carve(workspace, rows, true);
  if (workspace_bytes < w.bytes) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const __bf16* X = reinterpret_cast<const __bf16*>(x);
  const __bf16* Pb = reinterpret_cast<const __bf16*>(params_bf16);
  int rc = forward(rows, X, params, Pb, w.y, w, true, st);
  if (rc != VEC_OK) return rc;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(256), dim3(256), 0, st, grad, kParams);
  hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(loss),
                     (int64_t)2);
  hipLaunchKernelGGL(loss_kernel, dim3(256), dim3(256), 0, st, (int)rows, w.y, targets, colw,
                     scale, w.dy, loss);
  // backward: dZ of layer L is `dz` (BF16, rows x out_L); the layer's input
  // activation is `act`
  const int ksplit = rows >= 512 ? 512 : (int)rows;
  const int kz = (int)((rows + ksplit - 1) / ksplit);
  const __bf16* dz = w.dy;
  for (int L = 3; L >= 0; --L) {
    const int nin = kLayerIn[L], nout = kLayerOut[L];
    const __bf16* act = L == 0 ? X : w.h[L - 1];
    // dW_L = dZ^T act: M = nout, N = nin, K = rows (split, accumulated)
    GemmArgs gw = {};
    gw.M = nout;
    gw.N = nin;
    gw.k_begin = 0;
    gw.k_end = (int)rows;
    gw.k_split = ksplit;
    gw.A = dz;
    gw.lda = nout;
    gw.B = act;
    gw.ldb = nin;
    gw.C = grad + kOffW[L];
    gw.ldc = nin;
    if (gemm<true, false, kEpiAtomic>(gw, kz, st) != hipSuccess) return VEC_EHIP;
    hipLaunchKernelGGL(colsum_kernel, dim3((nout + 31) / 32), dim3(1024), 0, st, (int)rows, nout,
                       dz, grad + kOffB[L]);
    if (L == 0) break;
    // dZ_{L-1} = (dZ_L W_L) * silu'(Z_{L-1}): M = rows, N = nin, K = nout
    GemmArgs gb = {};
    gb.M = (int)rows;
    gb.N = nin;
    gb.k_begin = 0;
    gb.k_end = nout;
    gb.A = dz;
    gb.lda = nout;
    gb.B = Pb + kOffW[L];
    gb.ldb = nin;
    gb.Z = w.z[L - 1];
    gb.ldz = kHid;
    __bf16* out = w.dh[L & 1];
    gb.H = out;
    gb.ldh = kHid;
    if (gemm<false, false, kEpiBackAct>(gb, 1, st) != hipSuccess) return VEC_EHIP;
    dz = out;
  }
  return hip_rc(hipGetLastError());
}

int vec_mlp_adam(const float* grad, float* params, uint16_t* params_bf16, float* m1, float* m2,
                 int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!grad || !params || !params_bf16 || !m1 || !m2 || step < 1 || !(lr > 0.0f)) return VEC_EINVAL;
  const float c1 = 1.0f / (1.0f - powf(beta1, (float)step));
  const float c2 = 1.0f / (1.0f - powf(beta2, (float)step));
  hipLaunchKernelGGL(adam_kernel, dim3(256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     kParams, params, grad, m1, m2, reinterpret_cast<__bf16*>(params_bf16), lr,
                     beta1, beta2, eps, c1, c2);
  return hip_rc(hipGetLastError());
}

int vec_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* stream) {
  if (!params || !params_bf16) return VEC_EINVAL;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     kParams, params, reinterpret_cast<__bf16*>(params_bf16));
  return hip_rc(hipGetLastError());
}

int vec_surrogate_features(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                           const double* covparms, int64_t i0, int64_t i1, float dist_lo,
                           float dist_hi, uint16_t* features, uint8_t* flag, void* stream) {
  if (!pb || pb->family != VEC_FAMILY_ISO || pb->d != 2 || pb->m != kM) return VEC_EINVAL;
  if (i0 < 0 || i1 < i0 || i1 > pb->n || !locs || !NNarray || !covparms || !features)
    return VEC_EINVAL;
  const int64_t count = i1 - i0;
  if (count == 0) return VEC_OK;
  if ((reinterpret_cast<uintptr_t>(features) & 15) != 0) return VEC_EINVAL;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), i0, count, locs, NNarray, covparms,
                     pb->smoothness, dist_lo, dist_hi, reinterpret_cast<__bf16*>(features), flag);
  return hip_rc(hipGetLastError());
}

size_t vec_surrogate_workspace_bytes(const vec_problem* pb) {
  if (!pb || pb->p < 1 || pb->p > 3) return 0;
  const int nr = 2 + pb->p * pb->p + pb->p;
  return (size_t)1024 * nr * sizeof(double);
}

int vec_surrogate_sums(const vec_problem* pb, const int32_t* NNarray, const double* y,
                       const double* X, const double* covparms, int64_t i0, int64_t i1,
                       const float* pred, const uint8_t* flag, float lv_scale, float lv_shift,
                       float lv_slack, float lv_floor, double* raw, int32_t accumulate,
                       int32_t* back, uint32_t* nback, void* workspace, size_t workspace_bytes,
                       void* stream) {
  if (!pb || pb->family != VEC_FAMILY_ISO || pb->m != kM || pb->p < 1 || pb->p > 3)
    return VEC_EINVAL;
  if (i0 < 0 || i1 < i0 || i1 > pb->n || !NNarray || !y || !X || !covparms || !pred || !raw ||
      !back || !nback || (reinterpret_cast<uintptr_t>(pred) & 15) != 0)
    return VEC_EINVAL;
  if (!workspace || workspace_bytes < vec_surrogate_workspace_bytes(pb)) return VEC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t count = i1 - i0;
  const int nr = 2 + pb->p * pb->p + pb->p;
  int grid = (int)((count + 255) / 256);
  grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
  double* partials = static_cast<double*>(workspace);
  auto launch = [&](auto pc_) {
    constexpr int PC = decltype(pc_)::value;
    hipLaunchKernelGGL(sums_kernel<PC>, dim3(grid), dim3(256), 0, st, i0, count, NNarray,
                       y, X, covparms, pred, flag, lv_scale, lv_shift, lv_slack, lv_floor,
                       partials, back,
                       reinterpret_cast<unsigned int*>(nback));
  };
  if (pb->p == 1) launch(std::integral_constant<int, 1>{});
  else if (pb->p == 2) launch(std::integral_constant<int, 2>{});
  else launch(std::integral_constant<int, 3>{});
  hipLaunchKernelGGL(sum_rows_kernel, dim3(nr), dim3(256), 0, st, partials, grid, nr, raw,
                     accumulate);
  return hip_rc(hipGetLastError());
}

}  // extern "C"
