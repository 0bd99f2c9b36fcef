// Device kernels of the temporal-adaptive finite-volume path (gfx950).
//
// One subiteration of Alg. 2 (Sec. 2.2) on the device:
//   k_grad   (second order) cells that touch an active face: least-squares
//            gradient of the primitive variables over the 4 face neighbours
//            (mirror ghosts on the boundary), Barth-Jespersen limiter, and
//            the reconstructed value at each of the cell's 4 face centroids
//            (stored per half-face as [slot][variable][cell], so a face reads
//            2 x 5 values);
//   k_flux   once per face colour: active faces (faster side's level <= the
//            subiteration's level), exact Riemann flux, dt_f = 2^tau_f dt_min,
//            and a plain read-modify-write of both cells' FP64 accumulators;
//            no two faces of a colour share a cell, so no atomics and a fixed
//            summation order;
//   k_update cells whose level step ends: U += R / V, R = 0.
// At every iteration start (phase 0): k_dt (per-cell time step and its
// minimum), k_classify (levels from the dt ratio), k_sweep (neighbour
// levels at most one apart), and three ballot-based stable partitions that
// order faces by (colour, tau_f) and cells by tau_g / tau so that the
// active set of any subiteration is a prefix of each list.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "kernels.h"
#include "mlp.h"

namespace tafv {

constexpr int kBlock = 256;
constexpr int kCountSlots = kCounterSlots;
constexpr int kSlotStride = kCounterStride;  // 128 bytes between slots
constexpr int kPartChunk = 1024;  // elements per partition block (16 waves of 64)

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD works on one contiguous range of the list: its
// neighbour gathers then hit the L2 of that XCD.
__device__ inline int xcd_block() {
  int b = blockIdx.x, n = gridDim.x;
  int q = n >> 3;
  if (b < (q << 3)) return (b & 7) * q + (b >> 3);
  return b;
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// conserved (rho, m, E) -> primitive (rho, u, v, w, p)
__device__ inline void cons2prim(const double* U, double gm1, double* w) {
  double r = U[0], ir = 1.0 / r;
  double u = U[1] * ir, v = U[2] * ir, ww = U[3] * ir;
  w[0] = r;
  w[1] = u;
  w[2] = v;
  w[3] = ww;
  w[4] = gm1 * (U[4] - 0.5 * r * (u * u + v * v + ww * ww));
}

// ---------------------------------------------------------------------------
// state init and small fills

// prim in the caller's cell order; U, R in the internal order
__global__ void k_state_init(int nc, const int* __restrict__ perm, const double* __restrict__ prim,
                             double gm1, double* __restrict__ U, double* __restrict__ R) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double* w = prim + 5 * (size_t)perm[i];
  double r = w[0];
  U[5 * (size_t)i + 0] = r;
  U[5 * (size_t)i + 1] = r * w[1];
  U[5 * (size_t)i + 2] = r * w[2];
  U[5 * (size_t)i + 3] = r * w[3];
  U[5 * (size_t)i + 4] = w[4] / gm1 + 0.5 * r * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  for (int k = 0; k < 5; ++k) R[5 * (size_t)i + k] = 0.0;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// time step, classification, sweeps (phase 0 of an iteration)

// dt_i = cfl V_i / sum_f (|u_i . n_f| + a_i) |A_f|; dscal[0] <- min as bits
// (positive doubles order like their bit patterns); dscal[2] <- 1 on a
// non-physical state.
__global__ __launch_bounds__(kBlock) void k_dt(int nc, int nf, const double* __restrict__ U,
                                               const double* __restrict__ vol,
                                               const int* __restrict__ c2f,
                                               const double* __restrict__ fA, double gamma,
                                               double cfl, double* __restrict__ dt,
                                               unsigned long long* dscal) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double dti = INFINITY;
  if (i < nc) {
    double w[5];
    cons2prim(U + 5 * (size_t)i, gamma - 1.0, w);
    if (!(w[0] > 0.0) || !(w[4] > 0.0) || !isfinite(w[4])) {
      atomicOr(&dscal[2], 1ull);
    } else {
      double a = sqrt(gamma * w[4] / w[0]);
      double s = 0.0;
      for (int m = 0; m < 4; ++m) {
        int f = c2f[m * nc + i];
        double ax = fA[f], ay = fA[nf + f], az = fA[2 * (size_t)nf + f];
        double am = sqrt(ax * ax + ay * ay + az * az);
        double un = (w[1] * ax + w[2] * ay + w[3] * az) / am;
        s += (fabs(un) + a) * am;
      }
      dti = cfl * vol[i] / s;
    }
    dt[i] = dti;
  }
  __shared__ double smin[kBlock / 64];
  double v = wave_min(dti);
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = fmin(v, smin[k]);
    if (v < INFINITY) atomicMin(&dscal[0], (unsigned long long)__double_as_longlong(v));
  }
}

// tau_i = clamp(floor(log2(dt_i (1 - margin) / dt_min)), 0, L-1) by frexp
__global__ void k_classify(int nc, const double* __restrict__ dt, const unsigned long long* dscal,
                           double margin, int L, int8_t* __restrict__ lev) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  double dtmin = __longlong_as_double((long long)dscal[0]);
  double q = dt[i] * (1.0 - margin) / dtmin;
  int e;
  frexp(q, &e);
  int t = e - 1;
  t = t < 0 ? 0 : (t > L - 1 ? L - 1 : t);
  lev[i] = (int8_t)t;
}

// one lowering Jacobi sweep: tau_i <- min(tau_i, min_j tau_j + 1)
__global__ void k_sweep(int nc, const int* __restrict__ nb, const int8_t* __restrict__ src,
                        int8_t* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int t = src[i];
  for (int m = 0; m < 4; ++m) {
    int n = nb[m * nc + i];
    if (n >= 0) t = min(t, (int)src[n] + 1);
  }
  dst[i] = (int8_t)t;
}

// ---------------------------------------------------------------------------
// stable partition of indices by a small key, with wavefront ballots

struct ByteKey {
  const int8_t* key;
  __device__ int operator()(int i) const { return key[i]; }
};

// per face: tau_f = level of the faster side; key (colour, tau_f) or tau_f
__global__ void k_face_keys(int nf, const int* __restrict__ fhL, const int* __restrict__ fhR,
                            const int8_t* __restrict__ fcol, const int8_t* __restrict__ lev,
                            int use_colour, int8_t* __restrict__ fkey) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int t = lev[fhL[f] >> 2];
  int h = fhR[f];
  if (h >= 0) t = min(t, (int)lev[h >> 2]);
  fkey[f] = (int8_t)(use_colour ? fcol[f] * kMaxLevels + t : t);
}

// per cell: tau_g = lowest level of its faces (the partition key), the
// packed face word (tau_f per local face, higher-id side bits, tau), and
// the histogram hist[tau_g * 8 + tau] (block-local in LDS, then one atomic
// per bin and block)
__global__ __launch_bounds__(kBlock) void k_cell_keys(int nc, const int* __restrict__ nb,
                                                      const int8_t* __restrict__ lev,
                                                      int8_t* __restrict__ ckey,
                                                      uint32_t* __restrict__ fpack,
                                                      int* __restrict__ hist) {
  __shared__ int h[kMaxKeys];
  for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x) h[k] = 0;
  __syncthreads();
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) {
    int ti = lev[i], tg = ti;
    uint32_t pk = (uint32_t)ti << 20;
    for (int m = 0; m < 4; ++m) {
      int n = nb[m * nc + i];
      int tf = n >= 0 ? min(ti, (int)lev[n]) : ti;
      tg = min(tg, tf);
      pk |= (uint32_t)tf << (4 * m);
      if (n >= 0 && n < i) pk |= 1u << (16 + m);
    }
    ckey[i] = (int8_t)tg;
    fpack[i] = pk;
    atomicAdd(&h[tg * kMaxLevels + ti], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

// one buffer for the host readback at an iteration start: [0..5] the
// scalars (dt_min bits, theta slot, non-finite flag), [8..8+Kf] face list
// starts, [8+65..] cell list starts, [8+65+9..] the (tau_g, tau) histogram
__global__ void k_pack_readback(const unsigned long long* __restrict__ dscal,
                                const int* __restrict__ fstart, int Kf,
                                const int* __restrict__ cstart, const int* __restrict__ hist,
                                int* __restrict__ out) {
  int t = threadIdx.x;
  if (t < 6) out[t] = ((const int*)dscal)[t];
  if (t <= Kf) out[8 + t] = fstart[t];
  if (t <= kMaxLevels) out[8 + kMaxKeys + 1 + t] = cstart[t];
  if (t < kMaxKeys) out[8 + kMaxKeys + kMaxLevels + 2 + t] = hist[t];
}

hipError_t launch_pack_readback(hipStream_t s, DevMesh& m, int Kf) {
  hipLaunchKernelGGL(k_pack_readback, dim3(1), dim3(128), 0, s, m.dscal, m.pf.start, Kf,
                     m.pc.start, m.chist, m.rb);
  return hipGetLastError();
}

__global__ void k_fill_i32(int* p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename Key>
__global__ __launch_bounds__(64) void k_part_count(int n, Key key, int K, int nblocks,
                                                   int* __restrict__ counts) {
  __shared__ int cnt[kMaxKeys];
  int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) cnt[k] = 0;
  __syncthreads();
  int base = blockIdx.x * kPartChunk;
  for (int step = 0; step < kPartChunk / 64; ++step) {
    int i = base + step * 64 + lane;
    bool valid = i < n;
    int k_mine = valid ? key(i) : -1;
    unsigned long long pending = __ballot(valid);
    while (pending) {
      int leader = __ffsll(pending) - 1;
      int k = __shfl(k_mine, leader, 64);
      unsigned long long m = __ballot(k_mine == k);
      if (lane == leader) cnt[k] += __popcll(m);
      pending &= ~m;
    }
  }
  __syncthreads();
  for (int k = lane; k < K; k += 64) counts[k * nblocks + blockIdx.x] = cnt[k];
}

// start[k] = first slot of key k (offsets are scanned in (key, block) order)
__global__ void k_part_starts(int K, int nblocks, int n, const int* __restrict__ offs,
                              int* __restrict__ start) {
  int k = threadIdx.x;
  if (k < K) start[k] = offs[k * nblocks];
  if (k == K) start[K] = n;
}

// writes index i at slot pos of the partitioned list
struct IndexWriter {
  int* list;
  __device__ void operator()(int pos, int i, int) const { list[pos] = i; }
};

// writes the face record {f, hL, hR, tau_f}: the flux kernel then needs no
// second indirection
struct FaceWriter {
  int4* rec;
  const int* fhL;
  const int* fhR;
  __device__ void operator()(int pos, int f, int key) const {
    rec[pos] = make_int4(f, fhL[f], fhR[f], key & (kMaxLevels - 1));
  }
};

template <typename Key, typename Writer>
__global__ __launch_bounds__(64) void k_part_scatter(int n, Key key, int K, int nblocks,
                                                     const int* __restrict__ offs, Writer out) {
  __shared__ int base[kMaxKeys];
  int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) base[k] = offs[k * nblocks + blockIdx.x];
  __syncthreads();
  unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int first = blockIdx.x * kPartChunk;
  for (int step = 0; step < kPartChunk / 64; ++step) {
    int i = first + step * 64 + lane;
    bool valid = i < n;
    int k_mine = valid ? key(i) : -1;
    unsigned long long pending = __ballot(valid);
    while (pending) {
      int leader = __ffsll(pending) - 1;
      int k = __shfl(k_mine, leader, 64);
      unsigned long long m = __ballot(k_mine == k);
      int b0 = base[k];
      if (k_mine == k) out(b0 + __popcll(m & lt), i, k);
      __syncthreads();
      if (lane == leader) base[k] = b0 + __popcll(m);
      __syncthreads();
      pending &= ~m;
    }
  }
}

size_t partition_scan_bytes(int64_t n) {
  int nb = partition_blocks(n);
  size_t bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int*)nullptr, (int*)nullptr,
                                         kMaxKeys * nb);
  return bytes;
}

template <typename Key, typename Writer>
static hipError_t run_partition(hipStream_t s, int n, Key key, int K, Partition& p, Writer w) {
  int nb = partition_blocks(n);
  hipLaunchKernelGGL(k_part_count<Key>, dim3(nb), dim3(64), 0, s, n, key, K, nb, p.counts);
  size_t bytes = p.scan_bytes;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(p.scan_tmp, bytes, p.counts, p.offs, K * nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_starts, dim3(1), dim3(kMaxKeys + 1), 0, s, K, nb, n, p.offs, p.start);
  hipLaunchKernelGGL((k_part_scatter<Key, Writer>), dim3(nb), dim3(64), 0, s, n, key, K, nb,
                     p.offs, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// least-squares gradient + Barth-Jespersen limiter + face reconstruction

template <typename T>
struct GradArgs {
  const int* list;
  int count, nc, nf;
  const double* U;
  const int* nb;
  const T* lsq;  // [12][nc]
  const T* rf;   // [12][nc]
  const double* fA;
  T* Wf;  // [4][5][nc]
  double gm1;
  int boundary;
};

// Least squares over the 4 face neighbours (mirror ghosts on the boundary):
// G = sum_m c_m (W_m - W_i); Barth-Jespersen per variable k: the largest
// psi_k <= 1 keeping W_i + psi_k G_k . r_m inside [min, max] of the cell and
// its neighbours at all 4 face centroids r_m; output W_i + psi_k G_k . r_m.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_grad(GradArgs<T> a) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= a.count) return;
  const int nc = a.nc;
  int i = a.list[idx];
  double wd[5];
  cons2prim(a.U + 5 * (size_t)i, a.gm1, wd);
  T wi[5], dw[4][5];
  for (int k = 0; k < 5; ++k) wi[k] = (T)wd[k];
  for (int m = 0; m < 4; ++m) {
    int n = a.nb[m * nc + i];
    if (n >= 0) {
      double t[5];
      cons2prim(a.U + 5 * (size_t)n, a.gm1, t);
      for (int k = 0; k < 5; ++k) dw[m][k] = (T)t[k] - wi[k];
    } else {
      for (int k = 0; k < 5; ++k) dw[m][k] = 0;
      if (a.boundary == TAFV_BC_WALL) {
        int f = -n - 1;
        T ax = (T)a.fA[f], ay = (T)a.fA[a.nf + f], az = (T)a.fA[2 * (size_t)a.nf + f];
        T ia = frsq(ax * ax + ay * ay + az * az);
        T nx = ax * ia, ny = ay * ia, nz = az * ia;
        T un2 = 2 * (wi[1] * nx + wi[2] * ny + wi[3] * nz);
        dw[m][1] = -un2 * nx;
        dw[m][2] = -un2 * ny;
        dw[m][3] = -un2 * nz;
      }
    }
  }
  T r[4][3], c[4][3];
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 3; ++q) {
      r[m][q] = a.rf[(3 * m + q) * nc + i];
      c[m][q] = a.lsq[(3 * m + q) * nc + i];
    }
  T* __restrict__ out = a.Wf + i;  // [slot][variable][cell]
  for (int k = 0; k < 5; ++k) {
    T g0 = 0, g1 = 0, g2 = 0, hi = 0, lo = 0;
    for (int m = 0; m < 4; ++m) {
      T d = dw[m][k];
      g0 += c[m][0] * d;
      g1 += c[m][1] * d;
      g2 += c[m][2] * d;
      hi = d > hi ? d : hi;
      lo = d < lo ? d : lo;
    }
    T delta[4];
    T psi = 1;
    for (int m = 0; m < 4; ++m) {
      T d = g0 * r[m][0] + g1 * r[m][1] + g2 * r[m][2];
      delta[m] = d;
      T phi = 1;
      if (d > 0) phi = hi < d ? hi * frcp(d) : (T)1;
      else if (d < 0) phi = lo > d ? lo * frcp(d) : (T)1;
      psi = phi < psi ? phi : psi;
    }
    for (int m = 0; m < 4; ++m) out[(size_t)(5 * m + k) * nc] = wi[k] + psi * delta[m];
  }
}

// ---------------------------------------------------------------------------
// face flux

template <typename T>
struct FluxArgs {
  const int4* rec;  // active face records {f, hL, hR, tau_f}
  int count, nf, nc;
  const T* fA;      // [3][nf]
  const double* U;
  const T* Wf;
  double* R;        // colour scatter: accumulators
  double* Q;        // gather mode: per-face time-integrated flux [nf][5]
  unsigned long long* dcount;
  double* dimpulse;
  StepArgs s;
  // learned guess and face logging (kernels with features only)
  const MlpDev* mlp;
  float* log_rows;  // [log_cap][7]: 6 inputs, ln(p*/p_m)
  unsigned long long* log_count;
  long long log_cap;
  double log_rate;
  unsigned long long log_seed, subit;
  float guess_gate;
};

template <int ORDER, typename T>
__device__ inline void load_side(const FluxArgs<T>& a, int h, T* w) {
  if (ORDER == 2) {
    const T* p = a.Wf + (size_t)(5 * (h & 3)) * a.nc + (h >> 2);
    for (int k = 0; k < 5; ++k) w[k] = p[(size_t)k * a.nc];
  } else {
    double t[5];
    cons2prim(a.U + 5 * (size_t)(h >> 2), a.s.gas.gm1, t);
    for (int k = 0; k < 5; ++k) w[k] = (T)t[k];
  }
}

struct SolveInfo {
  int iters, fallback, vacuum;
  int gated, gated_iters, rejected, used;  // faces where two-rarefaction is inexact
};

// |A| F(W(0)) . n for one face: reconstructed states, rotation to the face
// normal, exact Riemann solve (p* in FP64), sampling at x/t = 0, flux.
template <int ORDER, typename T, bool G14>
__device__ inline void face_flux(const FluxArgs<T>& a, int4 r, T* phi, SolveInfo& info) {
  const Gas& G = a.s.gas;
  const int f = r.x, hL = r.y, hR = r.z;
  T ax = a.fA[f], ay = a.fA[a.nf + f], az = a.fA[2 * (size_t)a.nf + f];
  T wl[5], wr[5];
  load_side<ORDER, T>(a, hL, wl);
  if (hR >= 0) load_side<ORDER, T>(a, hR, wr);
  T a2 = ax * ax + ay * ay + az * az;
  T ia = frsq(a2);
  T am = a2 * ia;
  T nx = ax * ia, ny = ay * ia, nz = az * ia;
  T unl = wl[1] * nx + wl[2] * ny + wl[3] * nz;
  if (hR < 0 && a.s.boundary != TAFV_BC_WALL) {  // transmissive: F(W_L)
    T E = wl[4] * (T)(1.0 / G.gm1) + (T)0.5 * wl[0] * (wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
    phi[0] = am * wl[0] * unl;
    phi[1] = am * (wl[0] * unl * wl[1] + wl[4] * nx);
    phi[2] = am * (wl[0] * unl * wl[2] + wl[4] * ny);
    phi[3] = am * (wl[0] * unl * wl[3] + wl[4] * nz);
    phi[4] = am * unl * (E + wl[4]);
    return;
  }
  const bool wall = hR < 0;
  T unr = wall ? -unl : wr[1] * nx + wr[2] * ny + wr[3] * nz;
  const double rl = wl[0], pl = wl[4];
  const double rr = wall ? rl : (double)wr[0], pr = wall ? pl : (double)wr[4];
  Star st;
  double al, ar, ral, rar, ipl, ipr;
  if (G14) {
    double irl = frcp(rl), a2l = G.g * pl * irl;
    ral = frsq(a2l);
    al = a2l * ral;
    K14 KL = make_k14(G, pl, al, irl, ral);
    ipl = KL.ip;
    if (wall) {
      ar = al; rar = ral; ipr = ipl;
      st = solve_star14(G, unl, -(double)unl, al, al, KL, KL, a.s.newton_tol, a.s.newton_max_iter, -1.0);
    } else {
      double irr = frcp(rr), a2r = G.g * pr * irr;
      rar = frsq(a2r);
      ar = a2r * rar;
      K14 KR = make_k14(G, pr, ar, irr, rar);
      ipr = KR.ip;
      st = solve_star14(G, unl, unr, al, ar, KL, KR, a.s.newton_tol, a.s.newton_max_iter, -1.0);
    }
  } else {
    al = sqrt(G.g * pl / rl);
    ar = sqrt(G.g * pr / rr);
    ral = 1.0 / al; rar = 1.0 / ar; ipl = 1.0 / pl; ipr = 1.0 / pr;
    st = solve_star<false>(G, rl, unl, pl, al, rr, unr, pr, ar, a.s.newton_tol,
                           a.s.newton_max_iter, -1.0);
  }
  info.iters = st.iters;
  info.fallback = st.fallback;
  info.vacuum = st.vacuum;
  if (wall) {  // no mass or energy through a wall; the star pressure pushes
    T ps = (T)st.p;
    phi[0] = 0;
    phi[1] = ps * am * nx;
    phi[2] = ps * am * ny;
    phi[3] = ps * am * nz;
    phi[4] = 0;
    return;
  }
  T rs, us, ps;
  int side;
  if (G14 && !st.vacuum)
    side = sample14<T>(G, wl[0], unl, wl[4], (T)al, (T)ipl, (T)ral, wr[0], unr, wr[4], (T)ar,
                       (T)ipr, (T)rar, (T)st.p, (T)st.u, rs, us, ps);
  else
    side = sample0<G14, T>(G, wl[0], unl, wl[4], (T)al, wr[0], unr, wr[4], (T)ar, (T)st.p,
                           (T)st.u, st.vacuum, rs, us, ps);
  const T* ws = side ? wr : wl;
  T uns = side ? unr : unl;
  T vx = us * nx + (ws[1] - uns * nx);
  T vy = us * ny + (ws[2] - uns * ny);
  T vz = us * nz + (ws[3] - uns * nz);
  T E = ps * (T)(1.0 / G.gm1) + (T)0.5 * rs * (vx * vx + vy * vy + vz * vz);
  phi[0] = am * rs * us;
  phi[1] = am * (rs * us * vx + ps * nx);
  phi[2] = am * (rs * us * vy + ps * ny);
  phi[3] = am * (rs * us * vz + ps * nz);
  phi[4] = am * us * (E + ps);
}

// Counters are spread over kCountSlots slots 128 bytes apart (slot = block
// index modulo kCountSlots) so that the waves of a launch do not all
// serialise on one address; the host sums the slots.
__device__ inline void flush_counters(const SolveInfo& info, double i0, double i1, double i2,
                                      unsigned long long* dcount, double* dimpulse) {
  __shared__ int s_cnt[7];
  __shared__ double s_imp[3];
  if (threadIdx.x < 7) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x < 3) s_imp[threadIdx.x] = 0.0;
  __syncthreads();
  int c[7] = {wave_sum(info.iters), wave_sum(info.fallback), wave_sum(info.vacuum),
              wave_sum(info.gated), wave_sum(info.gated_iters), wave_sum(info.rejected),
              wave_sum(info.used)};
  i0 = wave_sum(i0);
  i1 = wave_sum(i1);
  i2 = wave_sum(i2);
  if ((threadIdx.x & 63) == 0) {
    for (int k = 0; k < 7; ++k)
      if (c[k]) atomicAdd(&s_cnt[k], c[k]);
    if (i0 != 0.0 || i1 != 0.0 || i2 != 0.0) {
      atomicAdd(&s_imp[0], i0);
      atomicAdd(&s_imp[1], i1);
      atomicAdd(&s_imp[2], i2);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* cs = dcount + (blockIdx.x % kCountSlots) * kSlotStride;
    for (int k = 0; k < 7; ++k)
      if (s_cnt[k]) atomicAdd(&cs[k], (unsigned long long)s_cnt[k]);
    if (s_imp[0] != 0.0 || s_imp[1] != 0.0 || s_imp[2] != 0.0) {
      double* d = dimpulse + (blockIdx.x % kCountSlots) * kSlotStride;
      atomicAdd(&d[0], s_imp[0]);
      atomicAdd(&d[1], s_imp[1]);
      atomicAdd(&d[2], s_imp[2]);
    }
  }
}

// Colour scatter: the faces of one colour share no cell, so each thread
// reads, updates and writes both cells' accumulators with plain memory
// operations.  The accumulators are loaded before the flux is computed so
// their latency overlaps the solve.
template <int ORDER, typename T, bool G14>
__global__ __launch_bounds__(kBlock) void k_flux_colour(FluxArgs<T> a) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  if (idx < a.count) {
    int4 r = a.rec[idx];
    int cL = r.y >> 2, cR = r.z >> 2;
    double* RL = a.R + 5 * (size_t)cL;
    double* RR = a.R + 5 * (size_t)(r.z >= 0 ? cR : cL);
    double accL[5], accR[5];
    for (int k = 0; k < 5; ++k) {
      accL[k] = RL[k];
      accR[k] = RR[k];
    }
    T phi[5];
    face_flux<ORDER, T, G14>(a, r, phi, info);
    double dtf = ldexp(a.s.dt_min, r.w);
    double q[5];
    for (int k = 0; k < 5; ++k) {
      q[k] = dtf * (double)phi[k];
      RL[k] = accL[k] - q[k];
    }
    if (r.z >= 0) {
      for (int k = 0; k < 5; ++k) RR[k] = accR[k] + q[k];
    } else if (a.s.boundary == TAFV_BC_WALL) {
      i0 = q[1];
      i1 = q[2];
      i2 = q[3];
    }
  }
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

// Gather mode: store the time-integrated flux of each active face; the
// cells add their faces afterwards (k_cell_gather).
template <int ORDER, typename T, bool G14>
__global__ __launch_bounds__(kBlock) void k_flux_store(FluxArgs<T> a) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  if (idx < a.count) {
    int4 r = a.rec[idx];
    T phi[5];
    face_flux<ORDER, T, G14>(a, r, phi, info);
    double dtf = ldexp(a.s.dt_min, r.w);
    double* q = a.Q + 5 * (size_t)r.x;
    for (int k = 0; k < 5; ++k) q[k] = dtf * (double)phi[k];
    if (r.z < 0 && a.s.boundary == TAFV_BC_WALL) {
      i0 = q[1];
      i1 = q[2];
      i2 = q[3];
    }
  }
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

// splitmix64 output function (Steele, Lea, Flood 2014): a counter-based
// hash for sampling the logged faces
__device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Gather-mode flux for gamma = 1.4 with the optional features:
//   FEAT & 1: statistics of the faces where the two-rarefaction start is
//             inexact (p_TR > min(p_L, p_R), at least one shock) and face
//             logging of a hashed sample of them (inputs and ln(p*/p_TR));
//   FEAT & 2: on those faces the network predicts y ~ ln(p*/p_TR); where
//             |y| exceeds the gate the Newton solve starts from p_TR exp(y)
//             (a non-finite or non-positive guess falls back to p_TR).  The
//             network runs once per wave, on the matrix cores, when any lane
//             of the wave needs it.
// The Newton iteration and its stop test are unchanged, so p* is the same
// root whichever start is used.
template <int ORDER, typename T, int FEAT>
__global__ __launch_bounds__(kBlock) void k_flux_feat(FluxArgs<T> a) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[(FEAT & 2) ? (kBlock / 64) * kMlpFwdLds : 8];
  const Gas& G = a.s.gas;
  int idx = xcd_block() * kBlock + threadIdx.x;
  const bool valid = idx < a.count;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  int4 r = valid ? a.rec[idx] : make_int4(0, 0, -1, 0);
  T wl[5] = {1, 0, 0, 0, 1}, wr[5] = {1, 0, 0, 0, 1};
  T am = 1, nx = 1, ny = 0, nz = 0, unl = 0, unr = 0;
  bool wall = false, transmit = false, vac = false, gate = false;
  double al = 1, ar = 1, ral = 1, rar = 1, ptr = -1.0, pm = 1.0;
  K14 KL{}, KR{};
  float x[kMlpIn] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    const int f = r.x;
    T ax = a.fA[f], ay = a.fA[a.nf + f], az = a.fA[2 * (size_t)a.nf + f];
    load_side<ORDER, T>(a, r.y, wl);
    wall = r.z < 0 && a.s.boundary == TAFV_BC_WALL;
    transmit = r.z < 0 && !wall;
    if (r.z >= 0) load_side<ORDER, T>(a, r.z, wr);
    T a2 = ax * ax + ay * ay + az * az;
    T ia = frsq(a2);
    am = a2 * ia;
    nx = ax * ia;
    ny = ay * ia;
    nz = az * ia;
    unl = wl[1] * nx + wl[2] * ny + wl[3] * nz;
    if (!transmit) {
      double rl = wl[0], pl = wl[4];
      double irl = frcp(rl), a2l = G.g * pl * irl;
      ral = frsq(a2l);
      al = a2l * ral;
      KL = make_k14(G, pl, al, irl, ral);
      if (wall) {
        unr = -unl;
        ar = al;
        rar = ral;
        KR = KL;
      } else {
        unr = wr[1] * nx + wr[2] * ny + wr[3] * nz;
        double rr = wr[0], pr = wr[4];
        double irr = frcp(rr), a2r = G.g * pr * irr;
        rar = frsq(a2r);
        ar = a2r * rar;
        KR = make_k14(G, pr, ar, irr, rar);
      }
      vac = G.two_gm1 * (al + ar) <= (double)unr - (double)unl;
      if (!vac) {
        double num = al + ar - 0.5 * G.gm1 * ((double)unr - (double)unl);
        double den = al * irt7(KL.p) + ar * irt7(KR.p);
        double q = num * frcp(den), q2 = q * q, q3 = q2 * q;
        ptr = q3 * q3 * q;
        gate = !wall && ptr > fmin(KL.p, KR.p);
      }
      if (gate) {
        double rr = wr[0];
        double rm = 0.5 * ((double)wl[0] + rr);
        pm = 0.5 * (KL.p + KR.p);
        double amean = sqrt(G.g * pm / rm);
        x[0] = (float)((double)wl[0] / rm);
        x[1] = (float)((double)unl / amean);
        x[2] = (float)(KL.p / pm);
        x[3] = (float)(rr / rm);
        x[4] = (float)((double)unr / amean);
        x[5] = (float)(KR.p / pm);
      }
    }
  }
  float ym = 0.f;
  if ((FEAT & 2) && __ballot(gate) != 0ull)
    ym = mlp_wave_forward(*a.mlp, x, lds + (threadIdx.x >> 6) * kMlpFwdLds);
  if (valid) {
    T phi[5];
    if (transmit) {
      T E = wl[4] * (T)(1.0 / G.gm1) + (T)0.5 * wl[0] * (wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
      phi[0] = am * wl[0] * unl;
      phi[1] = am * (wl[0] * unl * wl[1] + wl[4] * nx);
      phi[2] = am * (wl[0] * unl * wl[2] + wl[4] * ny);
      phi[3] = am * (wl[0] * unl * wl[3] + wl[4] * nz);
      phi[4] = am * unl * (E + wl[4]);
    } else {
      double guess = ptr;
      if ((FEAT & 2) && gate && fabsf(ym) > a.guess_gate) {
        double gm = ptr * exp((double)ym);
        if (gm > 0.0 && isfinite(gm)) {
          guess = gm;
          info.used = 1;
        } else {
          info.rejected = 1;
        }
      }
      Star st = solve_star14(G, unl, unr, al, ar, KL, KR, a.s.newton_tol, a.s.newton_max_iter,
                             guess);
      info.iters = st.iters;
      info.fallback = st.fallback;
      info.vacuum = st.vacuum;
      if (gate) {
        info.gated = 1;
        info.gated_iters = st.iters;
        if ((FEAT & 1) && a.log_cap > 0) {
          unsigned long long h = mix64(a.log_seed ^ mix64(((unsigned long long)r.x << 24) ^ a.subit));
          if ((double)(h >> 11) * 0x1.0p-53 < a.log_rate) {
            unsigned long long slot = atomicAdd(a.log_count, 1ull);
            if (slot < (unsigned long long)a.log_cap) {
              float* row = a.log_rows + 7 * slot;
              for (int k = 0; k < kMlpIn; ++k) row[k] = x[k];
              row[6] = (float)log(st.p / ptr);
            }
          }
        }
      }
      if (wall) {
        T ps = (T)st.p;
        phi[0] = 0;
        phi[1] = ps * am * nx;
        phi[2] = ps * am * ny;
        phi[3] = ps * am * nz;
        phi[4] = 0;
      } else {
        T rs, us, ps;
        int side;
        if (!st.vacuum)
          side = sample14<T>(G, wl[0], unl, wl[4], (T)al, (T)KL.ip, (T)ral, wr[0], unr, wr[4],
                             (T)ar, (T)KR.ip, (T)rar, (T)st.p, (T)st.u, rs, us, ps);
        else
          side = sample0<true, T>(G, wl[0], unl, wl[4], (T)al, wr[0], unr, wr[4], (T)ar, (T)st.p,
                                  (T)st.u, st.vacuum, rs, us, ps);
        const T* ws = side ? wr : wl;
        T uns = side ? unr : unl;
        T vx = us * nx + (ws[1] - uns * nx);
        T vy = us * ny + (ws[2] - uns * ny);
        T vz = us * nz + (ws[3] - uns * nz);
        T E = ps * (T)(1.0 / G.gm1) + (T)0.5 * rs * (vx * vx + vy * vy + vz * vz);
        phi[0] = am * rs * us;
        phi[1] = am * (rs * us * vx + ps * nx);
        phi[2] = am * (rs * us * vy + ps * ny);
        phi[3] = am * (rs * us * vz + ps * nz);
        phi[4] = am * us * (E + ps);
      }
    }
    double dtf = ldexp(a.s.dt_min, r.w);
    double* q = a.Q + 5 * (size_t)r.x;
    for (int k = 0; k < 5; ++k) q[k] = dtf * (double)phi[k];
    if (wall) {
      i0 = q[1];
      i1 = q[2];
      i2 = q[3];
    }
  }
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

// Gather mode, per cell with an active face or whose step ends: add the
// active faces' fluxes in local face order (-q where the cell is the lower
// id of the face, +q otherwise), then U += R / V, R = 0 for ending steps.
__global__ __launch_bounds__(kBlock) void k_cell_gather(int count, const int* __restrict__ list,
                                                        int nc, const uint32_t* __restrict__ fpack,
                                                        const int* __restrict__ c2f,
                                                        const double* __restrict__ Q,
                                                        const double* __restrict__ vol,
                                                        double* __restrict__ U,
                                                        double* __restrict__ R, int tau_s,
                                                        int tau_upd, unsigned long long* dscal) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  int i = list[idx];
  uint32_t pk = fpack[i];
  int ti = (pk >> 20) & 15;
  bool ends = ti <= tau_upd;
  bool touched = false;
  double acc[5] = {0, 0, 0, 0, 0};
  double* Ri = R + 5 * (size_t)i;
  for (int m = 0; m < 4; ++m) {
    if ((int)((pk >> (4 * m)) & 15) > tau_s) continue;
    if (!touched) {
      for (int k = 0; k < 5; ++k) acc[k] = Ri[k];
      touched = true;
    }
    const double* q = Q + 5 * (size_t)c2f[m * nc + i];
    if (pk & (1u << (16 + m))) {
      for (int k = 0; k < 5; ++k) acc[k] += q[k];
    } else {
      for (int k = 0; k < 5; ++k) acc[k] -= q[k];
    }
  }
  if (ends) {
    if (!touched)
      for (int k = 0; k < 5; ++k) acc[k] = Ri[k];
    double v = vol[i];
    bool bad = false;
    for (int k = 0; k < 5; ++k) {
      double u = U[5 * (size_t)i + k] + acc[k] / v;
      U[5 * (size_t)i + k] = u;
      Ri[k] = 0.0;
      bad |= !isfinite(u);
    }
    if (bad) atomicOr(&dscal[2], 1ull);
  } else if (touched) {
    for (int k = 0; k < 5; ++k) Ri[k] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// cells whose level step ends: U += R / V, R = 0

__global__ __launch_bounds__(kBlock) void k_update(int count, const int* __restrict__ list,
                                                   const int8_t* __restrict__ lev, int tau_upd,
                                                   const double* __restrict__ vol,
                                                   double* __restrict__ U, double* __restrict__ R,
                                                   unsigned long long* dscal) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  int i = list[idx];
  if (lev[i] > tau_upd) return;
  double v = vol[i];
  bool bad = false;
  for (int k = 0; k < 5; ++k) {
    double u = U[5 * (size_t)i + k] + R[5 * (size_t)i + k] / v;
    U[5 * (size_t)i + k] = u;
    R[5 * (size_t)i + k] = 0.0;
    bad |= !isfinite(u);
  }
  if (bad) atomicOr(&dscal[2], 1ull);
}

// caller-order staging: rows of `width` elements
template <typename T>
__global__ void k_rows_to_caller(int n, int width, const int* __restrict__ perm,
                                 const T* __restrict__ src, T* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < width; ++k) dst[(size_t)perm[i] * width + k] = src[(size_t)i * width + k];
}

template <typename T>
__global__ void k_rows_from_caller(int n, int width, const int* __restrict__ perm,
                                   const T* __restrict__ src, T* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < width; ++k) dst[(size_t)i * width + k] = src[(size_t)perm[i] * width + k];
}

// ---------------------------------------------------------------------------
// launchers

static inline int blocks_for(int64_t n, int bs = kBlock) { return (int)((n + bs - 1) / bs); }

int partition_blocks(int64_t n) { return (int)((n + kPartChunk - 1) / kPartChunk); }

hipError_t launch_state_init(hipStream_t s, DevMesh& m, const double* d_prim, double gamma) {
  hipLaunchKernelGGL(k_state_init, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.perm,
                     d_prim, gamma - 1.0, m.U, m.R);
  return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, unsigned long long v, int n) {
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(hipStream_t s, double* p, double v, int64_t n) {
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_dt(hipStream_t s, DevMesh& m, const StepArgs& a) {
  hipLaunchKernelGGL(k_dt, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.nf, m.U, m.vol,
                     m.c2f, m.fA, a.gas.g, a.cfl, m.dt, m.dscal);
  return hipGetLastError();
}

hipError_t launch_classify(hipStream_t s, DevMesh& m, const StepArgs& a) {
  hipLaunchKernelGGL(k_classify, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.dt,
                     m.dscal, a.level_margin, m.max_levels, m.lev);
  for (int k = 0; k < m.max_levels - 1; ++k) {
    hipLaunchKernelGGL(k_sweep, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.nb_, m.lev,
                       m.lev2);
    std::swap(m.lev, m.lev2);
  }
  return hipGetLastError();
}

hipError_t launch_partitions(hipStream_t s, DevMesh& m) {
  int use_colour = m.scatter == TAFV_SCATTER_COLOUR;
  int Kf = use_colour ? m.ncolours * kMaxLevels : kMaxLevels;
  hipLaunchKernelGGL(k_face_keys, dim3(blocks_for(m.nf)), dim3(kBlock), 0, s, m.nf, m.fhL, m.fhR,
                     m.fcol, m.lev, use_colour, m.fkey);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kMaxKeys), 0, s, m.chist, 0, kMaxKeys);
  hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.nb_, m.lev,
                     m.ckey, m.fpack, m.chist);
  hipError_t e = run_partition(s, m.nf, ByteKey{m.fkey}, Kf, m.pf, FaceWriter{m.frec, m.fhL, m.fhR});
  if (e != hipSuccess) return e;
  return run_partition(s, m.nc, ByteKey{m.ckey}, kMaxLevels, m.pc, IndexWriter{m.pc.list});
}

template <typename T>
static hipError_t rows_to_caller(hipStream_t s, DevMesh& m, int width, const T* src, T* dst) {
  hipLaunchKernelGGL((k_rows_to_caller<T>), dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc,
                     width, m.perm, src, dst);
  return hipGetLastError();
}
template <typename T>
static hipError_t rows_from_caller(hipStream_t s, DevMesh& m, int width, const T* src, T* dst) {
  hipLaunchKernelGGL((k_rows_from_caller<T>), dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc,
                     width, m.perm, src, dst);
  return hipGetLastError();
}
hipError_t launch_to_caller_f64(hipStream_t s, DevMesh& m, const double* src, double* dst) {
  return rows_to_caller<double>(s, m, 5, src, dst);
}
hipError_t launch_from_caller_f64(hipStream_t s, DevMesh& m, const double* src, double* dst) {
  return rows_from_caller<double>(s, m, 5, src, dst);
}
hipError_t launch_to_caller_i8(hipStream_t s, DevMesh& m, const int8_t* src, int8_t* dst) {
  return rows_to_caller<int8_t>(s, m, 1, src, dst);
}
hipError_t launch_from_caller_i8(hipStream_t s, DevMesh& m, const int8_t* src, int8_t* dst) {
  return rows_from_caller<int8_t>(s, m, 1, src, dst);
}

hipError_t launch_grad(hipStream_t s, DevMesh& m, const StepArgs& a, int count) {
  if (count <= 0) return hipSuccess;
  if (a.precision == TAFV_FP32_FLUX) {
    GradArgs<float> g{m.pc.list, count, m.nc, m.nf, m.U, m.nb_, m.lsq32, m.rf32, m.fA,
                      (float*)m.Wf, a.gas.gm1, a.boundary};
    hipLaunchKernelGGL(k_grad<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s, g);
  } else {
    GradArgs<double> g{m.pc.list, count, m.nc, m.nf, m.U, m.nb_, m.lsq, m.rf, m.fA,
                       (double*)m.Wf, a.gas.gm1, a.boundary};
    hipLaunchKernelGGL(k_grad<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s, g);
  }
  return hipGetLastError();
}

template <typename T, bool G14>
static void flux_launch(hipStream_t s, int order, int scatter, int count, const FluxArgs<T>& f) {
  dim3 g(blocks_for(count)), b(kBlock);
  if (scatter == TAFV_SCATTER_COLOUR) {
    if (order == 2) hipLaunchKernelGGL((k_flux_colour<2, T, G14>), g, b, 0, s, f);
    else hipLaunchKernelGGL((k_flux_colour<1, T, G14>), g, b, 0, s, f);
  } else {
    if (order == 2) hipLaunchKernelGGL((k_flux_store<2, T, G14>), g, b, 0, s, f);
    else hipLaunchKernelGGL((k_flux_store<1, T, G14>), g, b, 0, s, f);
  }
}

template <typename T>
static void flux_feat_launch(hipStream_t s, int order, int feat, int count, const FluxArgs<T>& f) {
  dim3 g(blocks_for(count)), b(kBlock);
#define TAFV_FEAT(O, F) hipLaunchKernelGGL((k_flux_feat<O, T, F>), g, b, 0, s, f)
  if (order == 2) {
    if (feat == 1) TAFV_FEAT(2, 1);
    else if (feat == 2) TAFV_FEAT(2, 2);
    else TAFV_FEAT(2, 3);
  } else {
    if (feat == 1) TAFV_FEAT(1, 1);
    else if (feat == 2) TAFV_FEAT(1, 2);
    else TAFV_FEAT(1, 3);
  }
#undef TAFV_FEAT
}

hipError_t launch_flux(hipStream_t s, DevMesh& m, const StepArgs& a, int first, int count,
                       const FluxFeatures& ft) {
  if (count <= 0) return hipSuccess;
  const int4* rec = m.frec + first;
  if (a.precision == TAFV_FP32_FLUX) {
    FluxArgs<float> f{rec, count, m.nf, m.nc, m.fA32, m.U, (const float*)m.Wf, m.R, m.Q, m.dcount,
                      m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                      ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate};
    if (ft.feat && a.gas.is14 && m.scatter == TAFV_SCATTER_GATHER)
      flux_feat_launch<float>(s, a.order, ft.feat, count, f);
    else if (a.gas.is14) flux_launch<float, true>(s, a.order, m.scatter, count, f);
    else flux_launch<float, false>(s, a.order, m.scatter, count, f);
  } else {
    FluxArgs<double> f{rec, count, m.nf, m.nc, m.fA, m.U, (const double*)m.Wf, m.R, m.Q,
                       m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                       ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate};
    if (ft.feat && a.gas.is14 && m.scatter == TAFV_SCATTER_GATHER)
      flux_feat_launch<double>(s, a.order, ft.feat, count, f);
    else if (a.gas.is14) flux_launch<double, true>(s, a.order, m.scatter, count, f);
    else flux_launch<double, false>(s, a.order, m.scatter, count, f);
  }
  return hipGetLastError();
}

hipError_t launch_cell_gather(hipStream_t s, DevMesh& m, int count, int tau_s, int tau_upd) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_gather, dim3(blocks_for(count)), dim3(kBlock), 0, s, count,
                     m.pc.list, m.nc, m.fpack, m.c2f, m.Q, m.vol, m.U, m.R, tau_s, tau_upd,
                     m.dscal);
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t s, DevMesh& m, int count, int tau_upd) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(blocks_for(count)), dim3(kBlock), 0, s, count, m.pc.list,
                     m.lev, tau_upd, m.vol, m.U, m.R, m.dscal);
  return hipGetLastError();
}

}  // namespace tafv
