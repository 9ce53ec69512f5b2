// Learned smoothness sensor: a 48 -> 64 -> 64 -> 1 network (GELU, sigmoid
// output) that predicts gamma_e from the cell features (see dgq_feat_kernel),
// on bfloat16 matrix cores (v_mfma_f32_32x32x16_bf16, float32 accumulation).
//
// Products are formed transposed, Z^T = W^T X^T, so that a wave's 32x32 tile
// holds one cell (or training sample) per lane column: lane l holds column
// l % 32 and, in accumulator v, row 8 (v / 4) + 4 (l / 32) + v % 4.  The
// second layer takes its B operand straight from the first layer's
// accumulators: the reduction index k of operand element i of lane group
// g = l / 32 is chosen as the row that group already holds (any k order
// gives the same sum, as long as A and B agree), so the A operand (W2^T)
// is read in two 4-element chunks.  No LDS round trip between the layers.
//
// Inference rounds inputs, weights and both hidden activations to bfloat16.
// Training keeps activations and back-propagated errors near float32 by
// splitting them into two bfloat16 terms (x = hi + lo, hi = bf16(x),
// lo = bf16(x - hi)) and summing the partial products on the matrix cores;
// weights and inputs are exact bfloat16 values.
#include "cvw_device.h"

namespace cvw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {    // 16-byte aligned
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}
__device__ __forceinline__ bf16x8 load4x2(const uint16_t* p0, const uint16_t* p1) {   // 8-byte aligned chunks
  const u32x2 a = *reinterpret_cast<const u32x2*>(p0), b = *reinterpret_cast<const u32x2*>(p1);
  u32x4 w;
  w[0] = a[0];
  w[1] = a[1];
  w[2] = b[0];
  w[3] = b[1];
  return __builtin_bit_cast(bf16x8, w);
}
__device__ __forceinline__ bf16x8 pack8(const uint16_t* h) {
  u32x4 w;
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = static_cast<uint32_t>(h[2 * q]) | (static_cast<uint32_t>(h[2 * q + 1]) << 16);
  return __builtin_bit_cast(bf16x8, w);
}
__device__ __forceinline__ bf16x8 zero8() {
  u32x4 w = {0u, 0u, 0u, 0u};
  return __builtin_bit_cast(bf16x8, w);
}
__device__ __forceinline__ f32x16 zero16() {
  f32x16 c;
#pragma unroll
  for (int v = 0; v < 16; ++v) c[v] = 0.0f;
  return c;
}
__device__ __forceinline__ f32x16 mma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// row of accumulator v for lane group g within a 32-row tile
__device__ __forceinline__ int acc_row(int v, int g) { return 8 * (v >> 2) + 4 * g + (v & 3); }

// erf(z) by the rational-exponential approximation of Abramowitz and Stegun,
// formula 7.1.26 (after Hastings): erf(z) = 1 - t (a1 + a2 t + ... + a5 t^4)
// exp(-z^2), t = 1 / (1 + p z), z >= 0, |error| <= 1.5e-7 (far below the
// bfloat16 rounding of the activations).  Also returns exp(-z^2).
__device__ __forceinline__ float erf_as(float z, float& ez) {
  const float az = fabsf(z);
  const float t = frcp(fmaf(0.3275911f, az, 1.0f));
  float q = fmaf(1.061405429f, t, -1.453152027f);
  q = fmaf(q, t, 1.421413741f);
  q = fmaf(q, t, -0.284496736f);
  q = fmaf(q, t, 0.254829592f);
  ez = __builtin_amdgcn_exp2f(-1.44269504088896341f * az * az);      // exp(-z^2) = 2^(-z^2 log2 e)
  const float y = fmaf(-q * t, ez, 1.0f);
  return z < 0.0f ? -y : y;
}
__device__ __forceinline__ float gelu(float x) {
  float e;
  return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f, e));
}
__device__ __forceinline__ float gelu_prime(float x) {
  float e;                                                            // e = exp(-x^2 / 2)
  const float ef = erf_as(x * 0.70710678118654752f, e);
  return fmaf(x * 0.39894228040143268f, e, 0.5f * (1.0f + ef));
}

// ---------------------------------------------------------------------------
// inference: 256 threads (4 waves), each wave one 32-cell tile per iteration
// ---------------------------------------------------------------------------
// With a guard G (learned sensor on a mesh): a cell whose features leave the
// network's validity box [lo, hi] (NaN included) or whose output is not
// finite, or every cell once the audit latch is set, gets gamma = NaN, its
// tile flag and a count: the plain sensor takes those cells over.
__global__ __launch_bounds__(256) void mlp_infer_kernel(const uint16_t* __restrict__ feat, int64_t n, MlpDev W,
                                                        float* __restrict__ gamma, MlpGuard G) {
  __shared__ float sb1[MLP_HID], sb2[MLP_HID], sw3[MLP_HID];
  __shared__ float slo[MLP_IN], shi[MLP_IN];
  // the weight operands of every lane, fragment-major (14 fragments x 64 lanes):
  // read per tile from LDS rather than held in registers
  __shared__ u32x4 sA[14][64];
  for (int t = threadIdx.x; t < MLP_HID; t += blockDim.x) {
    sb1[t] = W.b1[t];
    sb2[t] = W.b2[t];
    sw3[t] = bf16_value(W.w3[t]);
  }
  const bool guard = G.lo != nullptr;
  for (int t = threadIdx.x; t < MLP_IN; t += blockDim.x) {
    slo[t] = guard ? G.lo[t] : 0.0f;
    shi[t] = guard ? G.hi[t] : 0.0f;
  }
  const bool off = guard && G.status[WS_LEARNED_OFF] != 0u;
  for (int i = threadIdx.x; i < 14 * 64; i += blockDim.x) {
    const int f = i >> 6, l = i & 63, cl = l & 31, gl = l >> 5;
    bf16x8 a;
    if (f < 6) {
      const int ht = f / 3, kb = f % 3;
      a = load8(W.W1t + (32 * ht + cl) * MLP_IN + 16 * kb + 8 * gl);
    } else {
      const int ht = (f - 6) >> 2, st = ((f - 6) >> 1) & 1, kb = (f - 6) & 1;
      const uint16_t* row = W.W2t + (32 * ht + cl) * MLP_HID + 32 * st + 16 * kb + 4 * gl;
      a = load4x2(row, row + 8);
    }
    sA[f][l] = __builtin_bit_cast(u32x4, a);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, g = lane >> 5;
  const float b3 = W.b3[0];
  const int64_t ntiles = (n + 31) / 32;
  for (int64_t t = blockIdx.x * 4LL + wave; t < ntiles; t += static_cast<int64_t>(gridDim.x) * 4) {
    asm volatile("" ::: "memory");              // keeps the LDS weight reads in the loop
    const int64_t cell = t * 32 + c;
    const bool ok = cell < n;
    bf16x8 B1[3];
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) B1[kb] = ok ? load8(feat + cell * MLP_IN + 16 * kb + 8 * g) : zero8();
    // the lane's 24 features against the validity box (lane group g holds k = 16 kb + 8 g + i)
    bool outside = false;
    if (guard) {
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) {
        const u32x4 w = __builtin_bit_cast(u32x4, B1[kb]);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const uint16_t h = static_cast<uint16_t>((w[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
          const float x = bf16_value(h);
          const int k = 16 * kb + 8 * g + i;
          outside = outside || !(x >= slo[k] && x <= shi[k]);
        }
      }
    }
    f32x16 C1[2];
#pragma unroll
    for (int ht = 0; ht < 2; ++ht) {
      C1[ht] = zero16();
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) C1[ht] = mma(__builtin_bit_cast(bf16x8, sA[3 * ht + kb][lane]), B1[kb], C1[ht]);
    }
    bf16x8 B2[2][2];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        uint16_t h[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int v = 8 * kb + i;
          h[i] = bf16_bits(gelu(C1[st][v] + sb1[32 * st + acc_row(v, g)]));
        }
        B2[st][kb] = pack8(h);
      }
    float z = 0.0f;
#pragma unroll
    for (int ht = 0; ht < 2; ++ht) {
      f32x16 C2 = zero16();
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
          C2 = mma(__builtin_bit_cast(bf16x8, sA[6 + 4 * ht + 2 * st + kb][lane]), B2[st][kb], C2);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 32 * ht + acc_row(v, g);
        z = fmaf(sw3[r], bf16_value(bf16_bits(gelu(C2[v] + sb2[r]))), z);
      }
    }
    z += __shfl_xor(z, 32);
    float gv = 1.0f / (1.0f + expf(-(z + b3)));
    if (guard) {
      const bool other = __shfl_xor(static_cast<int>(outside), 32) != 0;
      const bool bad = ok && (off || outside || other || !isfinite(gv));
      if (bad) gv = __builtin_nanf("");
      if (bad && g == 0) {
        const int64_t i = cell % G.nx, j = cell / G.nx;
        G.tile_flag[(i / 16) + G.tiles_x * (j / 16)] = 1;
      }
      const unsigned long long m = __ballot(bad && g == 0);
      if (m && (threadIdx.x & 63) == __builtin_ctzll(m)) {
        atomicAdd(G.status + WS_FALLBACK_COUNT, static_cast<uint32_t>(__popcll(m)));
        atomicOr(G.status + WS_STATUS, ST_LEARNED_FALLBACK);
      }
    }
    if (g == 0 && ok) gamma[cell] = gv;
  }
}

// ---------------------------------------------------------------------------
// training: one wave per block, 32 samples; writes the block's gradient
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split(float x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_value(hi));
}

__global__ __launch_bounds__(64) void mlp_train_kernel(const uint16_t* __restrict__ feat,
                                                       const float* __restrict__ target,
                                                       const int32_t* __restrict__ idx, int batch, MlpDev W,
                                                       float* __restrict__ part) {
  __shared__ __align__(16) uint16_t sX[MLP_IN][32];
  __shared__ __align__(16) uint16_t sH1[2][MLP_HID][32];
  __shared__ __align__(16) uint16_t sD2[2][MLP_HID][32];
  __shared__ __align__(16) uint16_t sD1[2][MLP_HID][32];
  __shared__ float sD1f[MLP_HID][32], sD2f[MLP_HID][32], sH2f[MLP_HID][32], sd3[32];
  const int lane = threadIdx.x, c = lane & 31, g = lane >> 5;
  const int sglob = blockIdx.x * 32 + c;
  const bool ok = sglob < batch;
  const int64_t row = ok ? idx[sglob] : 0;
  float* out = part + static_cast<int64_t>(blockIdx.x) * MLP_NPARAM;

  // ---- forward ----
  bf16x8 B1[3];
#pragma unroll
  for (int kb = 0; kb < 3; ++kb) {
    B1[kb] = ok ? load8(feat + row * MLP_IN + 16 * kb + 8 * g) : zero8();
    const u32x4 w = __builtin_bit_cast(u32x4, B1[kb]);
#pragma unroll
    for (int i = 0; i < 8; ++i) sX[16 * kb + 8 * g + i][c] = static_cast<uint16_t>(w[i >> 1] >> (16 * (i & 1)));
  }
  float h1[2][16], gp1[2][16];
#pragma unroll
  for (int ht = 0; ht < 2; ++ht) {
    f32x16 C = zero16();
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) C = mma(load8(W.W1t + (32 * ht + c) * MLP_IN + 16 * kb + 8 * g), B1[kb], C);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float z = C[v] + W.b1[32 * ht + acc_row(v, g)];
      h1[ht][v] = gelu(z);
      gp1[ht][v] = gelu_prime(z);
    }
  }
  bf16x8 Bh[2][2], Bl[2][2];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      uint16_t hi[8], lo[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) split(h1[st][8 * kb + i], hi[i], lo[i]);
      Bh[st][kb] = pack8(hi);
      Bl[st][kb] = pack8(lo);
    }
  float h2[2][16], gp2[2][16];
  float z3 = 0.0f;
#pragma unroll
  for (int ht = 0; ht < 2; ++ht) {
    f32x16 C = zero16();
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const uint16_t* r = W.W2t + (32 * ht + c) * MLP_HID + 32 * st + 16 * kb + 4 * g;
        const bf16x8 A = load4x2(r, r + 8);
        C = mma(A, Bh[st][kb], C);
        C = mma(A, Bl[st][kb], C);
      }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int n2 = 32 * ht + acc_row(v, g);
      const float z = C[v] + W.b2[n2];
      h2[ht][v] = gelu(z);
      gp2[ht][v] = gelu_prime(z);
      z3 = fmaf(bf16_value(W.w3[n2]), h2[ht][v], z3);
    }
  }
  z3 += __shfl_xor(z3, 32);
  const float gam = 1.0f / (1.0f + expf(-(z3 + W.b3[0])));
  const float d3 = ok ? 2.0f * (gam - target[row]) / static_cast<float>(batch) * gam * (1.0f - gam) : 0.0f;

  // ---- backward ----
  float d2[2][16];
#pragma unroll
  for (int ht = 0; ht < 2; ++ht)
#pragma unroll
    for (int v = 0; v < 16; ++v) d2[ht][v] = d3 * bf16_value(W.w3[32 * ht + acc_row(v, g)]) * gp2[ht][v];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      uint16_t hi[8], lo[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) split(d2[st][8 * kb + i], hi[i], lo[i]);
      Bh[st][kb] = pack8(hi);
      Bl[st][kb] = pack8(lo);
    }
  float d1[2][16];
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    // d1 = (W2 d2) * gelu'(z1): A = W2 rows k, reduction over n in the held-row order
    f32x16 C = zero16();
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const uint16_t* r = W.W2r + (32 * kt + c) * MLP_HID + 32 * st + 16 * kb + 4 * g;
        const bf16x8 A = load4x2(r, r + 8);
        C = mma(A, Bh[st][kb], C);
        C = mma(A, Bl[st][kb], C);
      }
#pragma unroll
    for (int v = 0; v < 16; ++v) d1[kt][v] = C[v] * gp1[kt][v];
  }
  // transposed copies (row = unit, column = sample) for the weight gradients
#pragma unroll
  for (int ht = 0; ht < 2; ++ht)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 32 * ht + acc_row(v, g);
      uint16_t hi, lo;
      split(h1[ht][v], hi, lo);
      sH1[0][r][c] = hi;
      sH1[1][r][c] = lo;
      split(d2[ht][v], hi, lo);
      sD2[0][r][c] = hi;
      sD2[1][r][c] = lo;
      split(d1[ht][v], hi, lo);
      sD1[0][r][c] = hi;
      sD1[1][r][c] = lo;
      sD1f[r][c] = d1[ht][v];
      sD2f[r][c] = d2[ht][v];
      sH2f[r][c] = h2[ht][v];
    }
  if (g == 0) sd3[c] = d3;
  __syncthreads();
  // dW2[k][n] = sum_s h1[k][s] d2[n][s]
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 C = zero16();
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 Ah = load8(&sH1[0][32 * kt + c][16 * ks + 8 * g]), Al = load8(&sH1[1][32 * kt + c][16 * ks + 8 * g]);
        const bf16x8 Bh2 = load8(&sD2[0][32 * nt + c][16 * ks + 8 * g]), Bl2 = load8(&sD2[1][32 * nt + c][16 * ks + 8 * g]);
        C = mma(Ah, Bh2, C);
        C = mma(Ah, Bl2, C);
        C = mma(Al, Bh2, C);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) out[MLP_OFF_W2 + (32 * kt + acc_row(v, g)) * MLP_HID + 32 * nt + c] = C[v];
    }
  // dW1[f][k] = sum_s x[s][f] d1[k][s]
#pragma unroll
  for (int ft = 0; ft < 2; ++ft)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      f32x16 C = zero16();
      const int fr = 32 * ft + c;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 A = (fr < MLP_IN) ? load8(&sX[fr][16 * ks + 8 * g]) : zero8();
        C = mma(A, load8(&sD1[0][32 * kt + c][16 * ks + 8 * g]), C);
        C = mma(A, load8(&sD1[1][32 * kt + c][16 * ks + 8 * g]), C);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int f = 32 * ft + acc_row(v, g);
        if (f < MLP_IN) out[MLP_OFF_W1 + f * MLP_HID + 32 * kt + c] = C[v];
      }
    }
  // bias and output-weight gradients, fixed order over the 32 samples
  {
    float db1 = 0.0f, db2 = 0.0f, dw3 = 0.0f;
    for (int s = 0; s < 32; ++s) {
      db1 += sD1f[lane][s];
      db2 += sD2f[lane][s];
      dw3 = fmaf(sH2f[lane][s], sd3[s], dw3);
    }
    out[MLP_OFF_B1 + lane] = db1;
    out[MLP_OFF_B2 + lane] = db2;
    out[MLP_OFF_W3 + lane] = dw3;
    if (lane == 0) {
      float db3 = 0.0f;
      for (int s = 0; s < 32; ++s) db3 += sd3[s];
      out[MLP_OFF_B3] = db3;
    }
  }
}

// ---------------------------------------------------------------------------
// sum of the block gradients (float64, block order), Adam on the float32
// master weights (lr = 0: no update), and the compute copies
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_update_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ master, float* __restrict__ m1,
                                                         float* __restrict__ m2, float lr, float beta1, float beta2,
                                                         float omb1, float omb2, float eps, float bc1, float bc2,
                                                         float* __restrict__ grad_out, MlpDevMut W) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= MLP_NPARAM) return;
  double gs = 0.0;
  for (int b = 0; b < nblk; ++b) gs += static_cast<double>(part[static_cast<int64_t>(b) * MLP_NPARAM + j]);
  const float gr = static_cast<float>(gs);
  if (grad_out) grad_out[j] = gr;
  float w = master[j];
  if (lr > 0.0f) {
    const float a = beta1 * m1[j] + omb1 * gr;          // omb = 1 - beta, formed in float64
    const float b = beta2 * m2[j] + omb2 * gr * gr;
    m1[j] = a;
    m2[j] = b;
    w -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
    master[j] = w;
  }
  if (j < MLP_OFF_B1) {                      // W1[f][k]
    const int f = j / MLP_HID, k = j % MLP_HID;
    W.W1t[k * MLP_IN + f] = bf16_bits(w);
  } else if (j < MLP_OFF_W2) {
    W.b1[j - MLP_OFF_B1] = w;
  } else if (j < MLP_OFF_B2) {               // W2[k][n]
    const int q = j - MLP_OFF_W2, k = q / MLP_HID, n = q % MLP_HID;
    const uint16_t h = bf16_bits(w);
    W.W2t[n * MLP_HID + k] = h;
    W.W2r[k * MLP_HID + n] = h;
  } else if (j < MLP_OFF_W3) {
    W.b2[j - MLP_OFF_B2] = w;
  } else if (j < MLP_OFF_B3) {
    W.w3[j - MLP_OFF_W3] = bf16_bits(w);
  } else {
    W.b3[0] = w;
  }
}

// ---------------------------------------------------------------------------
cvw_status mlp_infer(const MlpDev& W, const uint16_t* feat, int64_t n, float* gamma, hipStream_t s,
                     const MlpGuard* guard) {
  if (n <= 0) return CVW_OK;
  const int64_t tiles = (n + 31) / 32;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((tiles + 3) / 4, 4096));
  const MlpGuard G = guard ? *guard : MlpGuard{};
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(grid), dim3(256), 0, s, feat, n, W, gamma, G);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status mlp_train(const MlpDev& W, const uint16_t* feat, const float* target, const int32_t* idx, int batch,
                     float* part, hipStream_t s) {
  const int nblk = (batch + 31) / 32;
  hipLaunchKernelGGL(mlp_train_kernel, dim3(nblk), dim3(64), 0, s, feat, target, idx, batch, W, part);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status mlp_update(const float* part, int nblk, float* master, float* m1, float* m2, float lr, double beta1,
                      double beta2, float eps, double bc1, double bc2, float* grad_out, const MlpDevMut& W,
                      hipStream_t s) {
  hipLaunchKernelGGL(mlp_update_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, part, nblk, master, m1, m2,
                     lr, static_cast<float>(beta1), static_cast<float>(beta2), static_cast<float>(1.0 - beta1),
                     static_cast<float>(1.0 - beta2), eps, static_cast<float>(bc1), static_cast<float>(bc2), grad_out,
                     W);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
