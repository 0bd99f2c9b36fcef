// The small network that proposes the initial star pressure of the exact
// Riemann solve (the learned guess), device side.
//
// Inputs per face (normal frame), deviations from the side averages
// rho_m, u_m, p_m normalised by them: x = (rho_L/rho_m - 1, (u_L - u_m)/a_m,
// p_L/p_m - 1, and the same for the right side), a_m = sqrt(g p_m / rho_m);
// network h1 = relu(W1 x + b1), h2 = relu(W2 h1 +
// b2) (32 units each), y = w3 . h2 + b3, a correction of the two-rarefaction
// value: guess p0 = p_TR exp(y).  BF16 inputs, weights and hidden
// activations (round to nearest even), FP32 accumulation.
//
// Matrix layer products run on v_mfma_f32_16x16x32_bf16: for a 16x32 A
// tile, a 32x16 B tile and a 16x16 FP32 result, lane l holds
//   A[l % 16][8 (l / 16) + v], B[8 (l / 16) + v][l % 16]  (v = 0..7),
//   D[4 (l / 16) + r][l % 16]                             (r = 0..3).
// A wave evaluates 64 rows: 4 row tiles x 2 column tiles per layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tafv {

constexpr int kMlpIn = 6;
constexpr int kMlpH = 32;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;  // 1313
// offsets in the parameter vector: W1 [32][6], b1, W2 [32][32], b2, w3, b3
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 224, kOffB2 = 1248, kOffW3 = 1280, kOffB3 = 1312;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Device copy of the network: BF16 weights packed as MFMA B fragments
// (lane-major, 16 bytes per lane), biases and the last layer as FP32 holding
// BF16-rounded values.
struct MlpDev {
  uint16_t w1f[2][64][8];   // layer 1: B[k][j] = W1[16c + j][k] (k < 6, else 0)
  uint16_t w2f[2][64][8];   // layer 2: B[k][j] = W2[16c + j][k]
  uint16_t w2tf[2][64][8];  // backward: B[j][k] = W2[j][16c + k]
  float b1[32], b2[32], w3[32], b3;
};

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ inline float bfround(float f) { return bf2f(f2bf(f)); }

struct U16x8 {
  uint16_t v[8];
};

__device__ inline bf16x8_t frag_contig(const uint16_t* p) {  // 16-byte aligned
  uint4 q = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8_t, q);
}
__device__ inline bf16x8_t frag_strided(const uint16_t* p, int stride) {
  U16x8 t;
  #pragma unroll
  for (int v = 0; v < 8; ++v) t.v[v] = p[v * stride];
  return __builtin_bit_cast(bf16x8_t, t);
}
__device__ inline bf16x8_t frag_global(const uint16_t* p) {
  uint4 q = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8_t, q);
}

__device__ inline f32x4_t mfma16(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// LDS per wave for the forward pass: X [64][8] then H [64][kHS]
constexpr int kHS = 40;  // padded row stride of hidden activations (elements)
constexpr int kMlpFwdLds = 64 * 8 + 64 * kHS;  // uint16 elements per wave

__device__ inline void lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward pass of one full wave (all 64 lanes must be active): lane l gives
// row l's inputs x[6] (FP32) and receives y.  lds: kMlpFwdLds uint16 of this
// wave, 16-byte aligned.  H1 is kept in LDS on request (training).
__device__ inline float mlp_wave_forward(const MlpDev& w, const float* x, uint16_t* lds,
                                         uint16_t* keep_h1 = nullptr) {
  const int l = threadIdx.x & 63, lo = l & 15, hi = l >> 4;
  uint16_t* X = lds;
  uint16_t* H = lds + 64 * 8;
  {
    U16x8 row;
    #pragma unroll
    for (int k = 0; k < 8; ++k) row.v[k] = k < kMlpIn ? f2bf(x[k]) : (uint16_t)0;
    *reinterpret_cast<uint4*>(X + 8 * l) = __builtin_bit_cast(uint4, row);
  }
  lds_order();
  const bf16x8_t zero = {};
  const bf16x8_t w1b0 = frag_global(&w.w1f[0][l][0]), w1b1 = frag_global(&w.w1f[1][l][0]);
  const bf16x8_t w2b0 = frag_global(&w.w2f[0][l][0]), w2b1 = frag_global(&w.w2f[1][l][0]);
  const float c10 = w.b1[lo], c11 = w.b1[16 + lo], c20 = w.b2[lo], c21 = w.b2[16 + lo];
  // layer 1: only k < 8 of the 32-deep product is non-zero (lanes 0..15)
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    bf16x8_t a = hi == 0 ? frag_contig(X + 8 * (16 * t + lo)) : zero;
    f32x4_t d0 = {c10, c10, c10, c10}, d1 = {c11, c11, c11, c11};
    d0 = mfma16(a, w1b0, d0);
    d1 = mfma16(a, w1b1, d1);
    #pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * t + 4 * hi + r;
      H[row * kHS + lo] = f2bf(fmaxf(d0[r], 0.f));
      H[row * kHS + 16 + lo] = f2bf(fmaxf(d1[r], 0.f));
    }
  }
  lds_order();
  if (keep_h1) {
    #pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<uint4*>(keep_h1 + l * kHS + 8 * q) =
          *reinterpret_cast<const uint4*>(H + l * kHS + 8 * q);
    lds_order();
  }
  // layer 2: a row tile is read (all 32 inputs) before it is overwritten
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    bf16x8_t a = frag_contig(H + (16 * t + lo) * kHS + 8 * hi);
    f32x4_t d0 = {c20, c20, c20, c20}, d1 = {c21, c21, c21, c21};
    d0 = mfma16(a, w2b0, d0);
    d1 = mfma16(a, w2b1, d1);
    lds_order();
    #pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * t + 4 * hi + r;
      H[row * kHS + lo] = f2bf(fmaxf(d0[r], 0.f));
      H[row * kHS + 16 + lo] = f2bf(fmaxf(d1[r], 0.f));
    }
    lds_order();
  }
  // layer 3: a dot product per row
  float y = w.b3;
  #pragma unroll
  for (int j = 0; j < kMlpH; ++j) y += bf2f(H[l * kHS + j]) * w.w3[j];
  return y;
}

}  // namespace tafv
