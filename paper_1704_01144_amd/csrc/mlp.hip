// Inference and training kernels of the learned p* guess (gfx950 MFMA).
//
// Training minimises the mean squared error of y ~ ln(p*/p_TR) over logged
// face states with Adam; FP32 master weights, BF16 copies for the
// MFMA products, FP32 accumulation.  One wave handles 64 rows per block:
//   forward  as mlp_wave_forward (keeping h1 and h2 in LDS);
//   backward dy = s (y - t) with s = 2 / batch,
//            dw3 = h2^T dy, db3 = sum dy, dz2 = dy w3^T * [h2 > 0],
//            dW2 = dz2^T h1, db2 = sum dz2   (MFMA, K = rows),
//            dh1 = dz2 W2                    (MFMA, K = 32),
//            dz1 = dh1 * [h1 > 0], dW1 = dz1^T x, db1 = sum dz1;
// each block writes its partial gradient; a second kernel sums the blocks
// in a fixed order, so a gradient is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "mlp.h"
#include "mlp_kernels.h"

namespace tafv {

// ---- packing FP32 parameters into the device network ---------------------

__global__ void k_mlp_pack(const float* __restrict__ th, MlpDev* __restrict__ w) {
  int t = threadIdx.x;  // 128 threads (2 column tiles x 64 lanes)
  int c = t >> 6, l = t & 63, lo = l & 15, hi = l >> 4;
  for (int v = 0; v < 8; ++v) {
    int k = 8 * hi + v;
    int j = 16 * c + lo;
    w->w1f[c][l][v] = k < kMlpIn ? f2bf(th[kOffW1 + j * kMlpIn + k]) : (uint16_t)0;
    w->w2f[c][l][v] = f2bf(th[kOffW2 + j * kMlpH + k]);
    // backward: B[j'][k'] = W2[j'][16c + k'] with j' = 8 hi + v, k' = lo
    w->w2tf[c][l][v] = f2bf(th[kOffW2 + k * kMlpH + j]);
  }
  if (t < kMlpH) {
    w->b1[t] = bfround(th[kOffB1 + t]);
    w->b2[t] = bfround(th[kOffB2 + t]);
    w->w3[t] = bfround(th[kOffW3 + t]);
  }
  if (t == 0) w->b3 = bfround(th[kOffB3]);
}

// ---- inference ----------------------------------------------------------

__global__ __launch_bounds__(64) void k_mlp_forward(int n, const float* __restrict__ x,
                                                    const MlpDev* __restrict__ w,
                                                    float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[kMlpFwdLds];
  int row = blockIdx.x * 64 + threadIdx.x;
  float xr[kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) xr[k] = row < n ? x[(size_t)row * kMlpIn + k] : 0.f;
  float out = mlp_wave_forward(*w, xr, lds);
  if (row < n) y[row] = out;
}

// ---- forward + backward over one minibatch -------------------------------

// rows of the batch: row i of [first, first + count) maps to data row
// (a * i + b) mod n (a coprime with n: a permutation of the data set)
struct BatchMap {
  unsigned long long a, b, n;
  long long first, count;
};

__global__ __launch_bounds__(64) void k_mlp_fwd_bwd(BatchMap bm, const float* __restrict__ x,
                                                    const float* __restrict__ tgt,
                                                    const MlpDev* __restrict__ w, float scale,
                                                    float* __restrict__ gpart,
                                                    float* __restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[kMlpFwdLds];
  __shared__ __attribute__((aligned(16))) uint16_t H1[64 * kHS];
  __shared__ __attribute__((aligned(16))) uint16_t DZ2[64 * kHS];
  __shared__ __attribute__((aligned(16))) uint16_t DZ1[64 * kHS];
  __shared__ float dyL[64];
  const int l = threadIdx.x, lo = l & 15, hi = l >> 4;
  long long i = (long long)blockIdx.x * 64 + l;
  bool valid = i < bm.count;
  unsigned long long row =
      valid ? (bm.a * (unsigned long long)(bm.first + i) + bm.b) % bm.n : 0ull;
  float xr[kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) xr[k] = valid ? x[row * kMlpIn + k] : 0.f;
  float y = mlp_wave_forward(*w, xr, lds, H1);
  const uint16_t* X = lds;
  const uint16_t* H2 = lds + 64 * 8;
  float t = valid ? tgt[row] : 0.f;
  float e = valid ? y - t : 0.f;
  float dy = scale * e;
  dyL[l] = dy;
  // dz2 = dy w3 * [h2 > 0]
  for (int j = 0; j < kMlpH; ++j) {
    float h2 = bf2f(H2[l * kHS + j]);
    DZ2[l * kHS + j] = f2bf(h2 > 0.f ? dy * w->w3[j] : 0.f);
  }
  lds_order();
  float* g = gpart + (size_t)blockIdx.x * kMlpParams;
  // last layer and the bias sums (lane j < 32 owns hidden unit j)
  if (l < kMlpH) {
    float gw3 = 0.f, gb2 = 0.f;
    for (int r = 0; r < 64; ++r) {
      gw3 += dyL[r] * bf2f(H2[r * kHS + l]);
      gb2 += bf2f(DZ2[r * kHS + l]);
    }
    g[kOffW3 + l] = gw3;
    g[kOffB2 + l] = gb2;
  }
  {
    float s = dy, q = e * e;
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_xor(s, off, 64);
      q += __shfl_xor(q, off, 64);
    }
    if (l == 0) {
      g[kOffB3] = s;
      lpart[blockIdx.x] = q;
    }
  }
  // dW2[j][k] = sum_rows dz2[row][j] h1[row][k]: M = j, N = k, K = rows
  #pragma unroll
  for (int mt = 0; mt < 2; ++mt)
    #pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x4_t d = {0.f, 0.f, 0.f, 0.f};
      #pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        int r0 = 32 * ks + 8 * hi;
        bf16x8_t a = frag_strided(DZ2 + r0 * kHS + 16 * mt + lo, kHS);
        bf16x8_t b = frag_strided(H1 + r0 * kHS + 16 * nt + lo, kHS);
        d = mfma16(a, b, d);
      }
      #pragma unroll
      for (int r = 0; r < 4; ++r)
        g[kOffW2 + (16 * mt + 4 * hi + r) * kMlpH + 16 * nt + lo] = d[r];
    }
  // dh1 = dz2 W2: M = rows, N = k, K = j; then dz1 = dh1 * [h1 > 0]
  const bf16x8_t wt0 = frag_global(&w->w2tf[0][l][0]), wt1 = frag_global(&w->w2tf[1][l][0]);
  #pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    bf16x8_t a = frag_contig(DZ2 + (16 * tt + lo) * kHS + 8 * hi);
    f32x4_t d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
    d0 = mfma16(a, wt0, d0);
    d1 = mfma16(a, wt1, d1);
    #pragma unroll
    for (int r = 0; r < 4; ++r) {
      int rr = 16 * tt + 4 * hi + r;
      float h0 = bf2f(H1[rr * kHS + lo]), h1v = bf2f(H1[rr * kHS + 16 + lo]);
      DZ1[rr * kHS + lo] = f2bf(h0 > 0.f ? d0[r] : 0.f);
      DZ1[rr * kHS + 16 + lo] = f2bf(h1v > 0.f ? d1[r] : 0.f);
    }
  }
  lds_order();
  if (l < kMlpH) {
    float gb1 = 0.f;
    for (int r = 0; r < 64; ++r) gb1 += bf2f(DZ1[r * kHS + l]);
    g[kOffB1 + l] = gb1;
  }
  // dW1[j][k] = sum_rows dz1[row][j] x[row][k]: M = j, N = k (< 6), K = rows
  #pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x4_t d = {0.f, 0.f, 0.f, 0.f};
    #pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      int r0 = 32 * ks + 8 * hi;
      bf16x8_t a = frag_strided(DZ1 + r0 * kHS + 16 * mt + lo, kHS);
      bf16x8_t b = lo < 8 ? frag_strided(X + r0 * 8 + lo, 8) : bf16x8_t{};
      d = mfma16(a, b, d);
    }
    if (lo < kMlpIn)
      #pragma unroll
      for (int r = 0; r < 4; ++r) g[kOffW1 + (16 * mt + 4 * hi + r) * kMlpIn + lo] = d[r];
  }
}

// grad[p] = sum over blocks in block order; loss = sum of the block losses
__global__ void k_mlp_reduce(int nblocks, const float* __restrict__ gpart,
                             const float* __restrict__ lpart, float* __restrict__ grad,
                             float* __restrict__ loss_acc, float loss_scale) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpParams) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += gpart[(size_t)b * kMlpParams + p];
    grad[p] = s;
  }
  if (p == kMlpParams) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += lpart[b];
    *loss_acc += s * loss_scale;
  }
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters, step count t >= 1
__global__ void k_mlp_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float gp = grad[p];
  float mp = b1 * m[p] + (1.f - b1) * gp;
  float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  th[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ void k_fill_f32(float* p, float val, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// ---- launchers ----------------------------------------------------------

hipError_t mlp_pack(hipStream_t s, const float* th, MlpDev* w) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(128), 0, s, th, w);
  return hipGetLastError();
}

hipError_t mlp_forward(hipStream_t s, int n, const float* x, const MlpDev* w, float* y) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + 63) / 64), dim3(64), 0, s, n, x, w, y);
  return hipGetLastError();
}

hipError_t mlp_gradient(hipStream_t s, unsigned long long a, unsigned long long b,
                        unsigned long long n, long long first, long long count, const float* x,
                        const float* t, const MlpDev* w, float* gpart, float* lpart, float* grad,
                        float* loss_acc, float loss_scale) {
  if (count <= 0) return hipSuccess;
  int nb = (int)((count + 63) / 64);
  BatchMap bm{a, b, n, first, count};
  hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(nb), dim3(64), 0, s, bm, x, t, w, 2.0f / (float)count,
                     gpart, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, nb,
                     gpart, lpart, grad, loss_acc, loss_scale);
  return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t s, float* th, float* m, float* v, const float* grad, float lr,
                    int step) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, th, m, v, grad,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_fill(hipStream_t s, float* p, float v, int n) {
  hipLaunchKernelGGL(k_fill_f32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace tafv
