// Device kernels of the temporal-adaptive finite-volume path (gfx950).
//
// One subiteration of Alg. 2 (Sec. 2.2) on the device, gather mode (the
// default):
//   k_grad         (second order) cells that touch an active face:
//                  least-squares gradient of the primitive variables over the
//                  4 face neighbours (mirror ghosts on the boundary),
//                  Barth-Jespersen limiter, and the reconstructed value at
//                  each of the cell's 4 face centroids (stored as
//                  [slot][cell][variable], so a face reads 2 runs of 5 values);
//   k_flux_store   active faces (faster side's level <= the subiteration's
//                  level): exact Riemann flux |A| F . n, stored per face;
//   k_cell_gather  cells with an active face or an ending step: the active
//                  faces' q = 2^tau_f dt_min Phi summed in local face order
//                  into the FP64 accumulator, U += R / V, R = 0 when the
//                  cell's level step ends (cells whose faces are all on their
//                  own level apply the whole step's sum at its start).
// Colour mode instead runs k_flux_colour once per face colour (a plain
// read-modify-write of both cells' accumulators; no two faces of a colour
// share a cell) and then k_update.  The predictor/corrector form adds
// k_predict and k_cell_gather2, a moving mesh k_face_speed and
// k_cell_gather_move.
// At every iteration start (phase 0): k_dt (per-cell time step and its
// minimum), k_classify_sweep (levels from the dt ratio and the first
// neighbour sweep), k_sweep_inplace (neighbour levels at most one apart),
// k_keys (face and cell keys, counted per block), k_cell_list_keys (the
// gather's key), k_part_scan and k_part_scatter (ballot-based stable
// partitions: faces by (colour, tau_f); cells by tau_g and, in the same pass,
// by the gather's key), so that the active set of any subiteration is a
// prefix, or a few ranges, of each list.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "kernels_dev.h"
#include "mlp.h"

namespace tafv {

constexpr int kPartChunk = 256;  // items per partition block (one wave, 64 items a step)
constexpr int kWholeMeshPct = 75;  // whole-mesh launches from this share of the cells on

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

// dmin[slot] <- min dt of the blocks of that slot, as bits (positive
// doubles order like their bit patterns; one slot per block modulo
// kCountSlots, so that the blocks' atomics do not serialise on one address);
// dscal[2] <- 1 on a non-physical state.
__global__ __launch_bounds__(kBlock) void k_dt(int nc, int nf, const double* __restrict__ U,
                                               const double* __restrict__ vol,
                                               const int* __restrict__ c2f,
                                               const double* __restrict__ fA, double gamma,
                                               double cfl, double* __restrict__ dt,
                                               unsigned long long* dscal,
                                               unsigned long long* dmin,
                                               const double* __restrict__ sF) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double dti = INFINITY;
  if (i < nc) {
    bool bad = false;
    dti = dt_item(i, nc, nf, U, vol, c2f, fA, gamma, cfl, bad, sF);
    if (bad) atomicOr(&dscal[2], 1ull);
    dt[i] = dti;
  }
  __shared__ double smin[kBlock / 64];
  double v = wave_min(dti);
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = fmin(v, smin[k]);
    if (v < INFINITY)
      atomicMin(&dmin[(blockIdx.x % kCountSlots) * kSlotStride],
                (unsigned long long)__double_as_longlong(v));
  }
}

// dscal[0] <- the minimum over the slots (one wave), which are set back to
// +inf for the next classification; the sweep flags and the level histogram
// of this classification start at zero
__global__ void k_min_slots(unsigned long long* __restrict__ dmin, unsigned long long* dscal,
                            unsigned* __restrict__ sweepf, int* __restrict__ chist) {
  unsigned long long v = dmin[threadIdx.x * kSlotStride];
  dmin[threadIdx.x * kSlotStride] = 0x7ff0000000000000ull;
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  if (threadIdx.x == 0) dscal[0] = v;
  if (threadIdx.x < kMaxLevels) sweepf[threadIdx.x] = 0u;
  for (int k = threadIdx.x; k < kCountSlots * kMaxKeys; k += 64) chist[k] = 0;
}

// Levels from the time steps, with the first lowering sweep taken at once
// (a Jacobi sweep: the neighbours' levels are classified from their own time
// steps): tau_i <- min(tau_i, tau_j + 1); changed[0] marks a lowered level.
__global__ __launch_bounds__(kBlock) void k_classify_sweep(int nc, const double* __restrict__ dt,
                                                           const unsigned long long* dscal,
                                                           double margin, int L,
                                                           const int* __restrict__ nb,
                                                           int8_t* __restrict__ lev,
                                                           unsigned* changed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool low = false;
  if (i < nc) {
    const double dtmin = __longlong_as_double((long long)dscal[0]);
    int n[4];
    double dn[4];
    for (int m = 0; m < 4; ++m) n[m] = nb[m * nc + i];
    for (int m = 0; m < 4; ++m) dn[m] = dt[n[m] >= 0 ? n[m] : i];
    const int t0 = classify_item(dt[i], dtmin, margin, L);
    int t = t0;
    for (int m = 0; m < 4; ++m)
      if (n[m] >= 0) t = min(t, classify_item(dn[m], dtmin, margin, L) + 1);
    lev[i] = (int8_t)t;
    low = t < t0;
  }
  if (__ballot(low) != 0ull && (threadIdx.x & 63) == 0) changed[0] = 1u;
}

// One lowering sweep in place, tau_i <- min(tau_i, tau_j + 1): a neighbour
// read while it is being lowered gives its old or its new level, both at or
// above the final one, so the levels after L-1 sweeps are the Jacobi
// sweeps' (the largest levels below the classification with neighbours at
// most one apart).  A sweep that lowers nothing has reached them: the next
// sweeps return at once (changed[k] marks sweep k lowering a level).
__global__ void k_sweep_inplace(int nc, const int* __restrict__ nb, int8_t* lev,
                                unsigned* changed, int k) {
  if (k > 0 && changed[k - 1] == 0u) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool low = false;
  if (i < nc) {
    int n[4], tn[4];
    for (int m = 0; m < 4; ++m) n[m] = nb[m * nc + i];
    for (int m = 0; m < 4; ++m) tn[m] = lev[n[m] >= 0 ? n[m] : i];
    const int t0 = lev[i];
    int t = t0;
    for (int m = 0; m < 4; ++m)
      if (n[m] >= 0) t = min(t, tn[m] + 1);
    if (t < t0) {
      lev[i] = (int8_t)t;
      low = true;
    }
  }
  if (__ballot(low) != 0ull && (threadIdx.x & 63) == 0) changed[k] = 1u;
}

// ---------------------------------------------------------------------------
// stable partition of indices by a small key, with wavefront ballots

// adds one wave's keys (k_mine < 0: no item) to the block's counters (LDS
// atomics: the waves of a block count into the same bins)
__device__ inline void block_count_keys(int* cnt, bool valid, int k_mine) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(valid);
  while (pending) {
    int leader = __ffsll(pending) - 1;
    int k = __shfl(k_mine, leader, 64);
    unsigned long long m = __ballot(valid && k_mine == k);
    if (lane == leader) atomicAdd(&cnt[k], __popcll(m));
    pending &= ~m;
  }
}

// Keys of one classification, one item per thread, with the partition
// counts of each block of kPartChunk (= kBlock) items: blocks [0, nbf) take
// the faces (tau_f, (colour, tau_f), or tau_f + 8 flocal) into
// fcounts[key][block]; blocks
// [nbf, nbf + nbc) the cells: tau_g and the packed face word, the
// (tau_g, tau) histogram, and, unless the gather's list is built too
// (count_cells = 0; k_cell_list_keys then counts both cell keys), the tau_g
// counts into ccounts[key][block].
__global__ __launch_bounds__(kBlock) void k_keys(int nf, int nbf, const int* __restrict__ fhL,
                                                 const int* __restrict__ fhR,
                                                 const int8_t* __restrict__ fcol, int use_colour,
                                                 const int8_t* __restrict__ flocal,
                                                 int Kf, int8_t* __restrict__ fkey,
                                                 int* __restrict__ fcounts, int nc, int nbc,
                                                 const int* __restrict__ nb,
                                                 const int8_t* __restrict__ lev,
                                                 int8_t* __restrict__ ckey,
                                                 uint32_t* __restrict__ fpack,
                                                 int* __restrict__ hist, int count_cells,
                                                 int* __restrict__ ccounts) {
  __shared__ int cnt[kMaxKeys];
  __shared__ int h[kMaxKeys];
  for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x) cnt[k] = h[k] = 0;
  __syncthreads();
  if ((int)blockIdx.x < nbf) {
    const int f = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = f < nf;
    int key = -1;
    if (valid) {
      key = face_key_item(f, fhL, fhR, fcol, lev, use_colour);
      if (flocal) key += kMaxLevels * flocal[f];
      fkey[f] = (int8_t)key;
    }
    block_count_keys(cnt, valid, key);
    __syncthreads();
    for (int k = threadIdx.x; k < Kf; k += blockDim.x) fcounts[k * nbf + blockIdx.x] = cnt[k];
    return;
  }
  const int b = blockIdx.x - nbf;
  const int i = b * kBlock + threadIdx.x;
  const bool valid = i < nc;
  const int bin = valid ? cell_key_item(i, nc, nb, lev, ckey, fpack) : 0;
  wave_hist_add(h, valid, bin);
  if (count_cells) block_count_keys(cnt, valid, valid ? bin / kMaxLevels : -1);
  __syncthreads();
  int* hs = hist + (b % kCountSlots) * kMaxKeys;
  for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x)
    if (h[k]) atomicAdd(&hs[k], h[k]);
  if (count_cells)
    for (int k = threadIdx.x; k < kMaxLevels; k += blockDim.x) ccounts[k * nbc + b] = cnt[k];
}

// cells that apply their fluxes at their step's start (kEarlyBit; order 0
// marks none) and the key of the gather's cell list: 2 tau for those cells,
// 2 tau_g + 1 for the others; with the partition counts of both cell keys
// per block, tau_g in ccounts[0..7][block], the gather's key in
// ccounts[8..23][block]
__global__ __launch_bounds__(kBlock) void k_cell_list_keys(int nc, int nbc,
                                                           const int* __restrict__ nb,
                                                           const int8_t* __restrict__ lev,
                                                           const int8_t* __restrict__ ckey,
                                                           uint32_t* __restrict__ fpack,
                                                           int8_t* __restrict__ lkey, int order,
                                                           int* __restrict__ ccounts) {
  __shared__ int cnt[kMaxLevels + kCellKeys];
  for (int k = threadIdx.x; k < kMaxLevels + kCellKeys; k += blockDim.x) cnt[k] = 0;
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < nc;
  int k1 = -1, k2 = -1;
  if (valid) {
    const bool e = cell_early_item(i, nc, nb, lev, ckey, fpack, order);
    k1 = ckey[i];
    k2 = e ? 2 * lev[i] : 2 * k1 + 1;
    lkey[i] = (int8_t)k2;
  }
  block_count_keys(cnt, valid, k1);
  block_count_keys(cnt, valid, valid ? kMaxLevels + k2 : -1);
  __syncthreads();
  for (int k = threadIdx.x; k < kMaxLevels + kCellKeys; k += blockDim.x)
    ccounts[k * nbc + blockIdx.x] = cnt[k];
}

// One buffer for the host readback at an iteration start: [0..5] the
// scalars (dt_min bits, theta slot, non-finite flag), [8..8+Kf] face list
// starts, [8+65..] cell list starts, [8+65+9..] the gather list's starts,
// then the (tau_g, tau) histogram.  Written by one block after both lists
// have their starts.
struct Readback {
  const unsigned long long* dscal;
  const int* fstart;
  int Kf;
  const int* cstart;
  const int* gstart;  // nullptr without the gather's list
  const int* hist;
  int* out;
};

__device__ inline void pack_readback(const Readback& r) {
  for (int t = threadIdx.x; t <= kMaxKeys; t += blockDim.x) {
    if (t < 6) r.out[t] = ((const int*)r.dscal)[t];
    if (t <= r.Kf) r.out[kRbFace + t] = r.fstart[t];
    if (t <= kMaxLevels) r.out[kRbCell + t] = r.cstart[t];
    if (t <= kCellKeys) r.out[kRbGather + t] = r.gstart ? r.gstart[t] : 0;
    if (t < kMaxKeys) {
      int sum = 0;
      for (int sl = 0; sl < kCountSlots; ++sl) sum += r.hist[sl * kMaxKeys + t];
      r.out[kRbHist + t] = sum;
    }
  }
}

__global__ void k_fill_i32(int* p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Stable partitions of an index range [0, n) by byte keys.  The key kernels
// count each block's (kPartChunk items) keys into counts[key][block];
// k_part_scan turns every key's row of counts into offsets within the row
// and a row total; the scatter adds the total of the keys before (so the
// list holds the keys in order) and writes each item at its slot, so the
// items of one key keep their index order.  Two keys over the same range (the
// two cell lists) share one pass: the second key's counts follow the
// first's ([K1 + K2][nblocks]) and its slots therefore start at n.

// writes one wave's items at base[key] onwards in lane order; the writer is
// given the slot less pofs and the key less kofs
template <typename Writer>
__device__ inline void wave_scatter_keys(int* base, bool valid, int k_mine, int i, int kofs,
                                         int pofs, const Writer& out) {
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long pending = __ballot(valid);
  while (pending) {
    int leader = __ffsll(pending) - 1;
    int k = __shfl(k_mine, leader, 64);
    unsigned long long m = __ballot(k_mine == k);
    int b0 = base[k];
    if (k_mine == k) out(b0 + __popcll(m & lt) - pofs, i, k - kofs);
    __syncthreads();
    if (lane == leader) base[k] = b0 + __popcll(m);
    __syncthreads();
    pending &= ~m;
  }
}

// One block per key row (blocks [0, Kf) the face partition's rows, the rest
// the cell partition's): the exclusive scan of the row's counts and the row
// total.  The row goes through LDS in tiles (coalesced loads and stores);
// in a tile each thread sums a run of consecutive entries, the threads'
// sums are scanned across the block, and the runs are rewritten in place.
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 8192;
__global__ __launch_bounds__(kScanThreads) void k_part_scan(int Kf, int nbf,
                                                            const int* __restrict__ fcounts,
                                                            int* __restrict__ foffs,
                                                            int* __restrict__ ftot, int nbc,
                                                            const int* __restrict__ ccounts,
                                                            int* __restrict__ coffs,
                                                            int* __restrict__ ctot) {
  __shared__ int tile[kScanTile];
  __shared__ int wsum[kScanThreads / 64];
  __shared__ int tile_end;
  const bool face = (int)blockIdx.x < Kf;
  const int k = face ? blockIdx.x : blockIdx.x - Kf;
  const int nb = face ? nbf : nbc;
  const int* in = (face ? fcounts : ccounts) + (size_t)k * nb;
  int* out = (face ? foffs : coffs) + (size_t)k * nb;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int carry = 0;
  for (int t0 = 0; t0 < nb; t0 += kScanTile) {
    const int n = min(kScanTile, nb - t0);
    for (int j = t; j < n; j += kScanThreads) tile[j] = in[t0 + j];
    __syncthreads();
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b0 = min(t * per, n), b1 = min(b0 + per, n);
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += tile[b];
    // exclusive scan of the thread sums: within the wave, then over the waves
    int inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
      int y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
      int x = lane < kScanThreads / 64 ? wsum[lane] : 0, xi = x;
      for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(xi, off, 64);
        if (lane >= off) xi += y;
      }
      if (lane < kScanThreads / 64) wsum[lane] = xi - x;  // exclusive over the waves
    }
    __syncthreads();
    int run = carry + wsum[w] + inc - sum;
    for (int b = b0; b < b1; ++b) {
      const int c = tile[b];
      tile[b] = run;
      run += c;
    }
    // the running total after this tile: the last thread's run end
    if (t == kScanThreads - 1) tile_end = run;
    __syncthreads();
    for (int j = t; j < n; j += kScanThreads) out[t0 + j] = tile[j];
    carry = tile_end;
    __syncthreads();
  }
  if (t == 0) (face ? ftot : ctot)[k] = carry;
}

// base[k] <- the first slot of key k: the row totals of the keys before it
// (tot has K <= 64 entries; one wave)
__device__ inline void key_starts(const int* __restrict__ tot, int K, int* start) {
  const int lane = threadIdx.x;
  if (lane >= 64) return;
  int x = lane < K ? tot[lane] : 0, xi = x;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(xi, off, 64);
    if (lane >= off) xi += y;
  }
  if (lane < K) start[lane] = xi - x;
}

// Block 0 also writes each list's key starts (start[k] = first slot of key
// k, start[K] = n), which the host reads back, and, given rb.out, packs the
// readback buffer.
template <typename Key, typename W1, typename W2>
__global__ __launch_bounds__(64) void k_part_scatter(int n, Key key1, int K1, W1 out1,
                                                     int* __restrict__ start1, Key key2, int K2,
                                                     W2 out2, int* __restrict__ start2,
                                                     int nblocks, const int* __restrict__ offs,
                                                     const int* __restrict__ tot, Readback rb) {
  __shared__ int ks[kMaxKeys];
  __shared__ int base[kMaxKeys];
  const int lane = threadIdx.x, K = K1 + K2;
  key_starts(tot, K, ks);
  __syncthreads();
  for (int k = lane; k < K; k += 64) base[k] = ks[k] + offs[k * nblocks + blockIdx.x];
  if (blockIdx.x == 0) {
    for (int k = lane; k < K1; k += 64) start1[k] = ks[k];
    for (int k = lane; k < K2; k += 64) start2[k] = ks[K1 + k] - n;
    if (lane == 0) start1[K1] = n;
    if (lane == 0 && K2 > 0) start2[K2] = n;
  }
  __syncthreads();
  const int first = blockIdx.x * kPartChunk;
  for (int step = 0; step < kPartChunk / 64; ++step) {
    const int i = first + step * 64 + lane;
    const bool valid = i < n;
    wave_scatter_keys(base, valid, valid ? key1(i) : -1, i, 0, 0, out1);
    if (K2 > 0) wave_scatter_keys(base, valid, valid ? K1 + key2(i) : -1, i, K1, n, out2);
  }
  if (blockIdx.x == 0 && rb.out) {
    __threadfence_block();
    __syncthreads();
    pack_readback(rb);
  }
}

// ---------------------------------------------------------------------------
// least-squares gradient + Barth-Jespersen limiter + face reconstruction

// Each wave stages its face values in LDS for coalesced stores (see
// FaceValueWriter); neighbour states are read through the global gather.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_grad(GradArgs<T> a) {
  __shared__ T sStage[kBlock / 64][kStageVals];
  const int b0 = a.first + xcd_block() * kBlock;
  const int idx = b0 + threadIdx.x;
  const int w0 = b0 + (threadIdx.x & ~63);  // the wave's first item
  if (w0 >= a.count) return;                // the whole wave is past the end
  if (a.list) {
    const bool valid = idx < a.count;
    grad_item<T>(a, list_cell(a.list, a.n1, a.off2, valid ? idx : w0), valid,
                 sStage[threadIdx.x >> 6]);
    return;
  }
  // whole mesh in its own order: cells outside the key range are skipped.
  // A lane requests its cell's own data together with the cell's key (one
  // trip to memory for both); a lane out of range computes its cell and
  // stores nothing.
  const int ic = idx < a.count ? idx : a.count - 1;
  const GradIn<T> g = grad_load<T>(a, ic);
  const bool in = idx < a.count && a.key[idx] <= a.key_max;
  if (__ballot(in) == 0ull) return;  // the wave has no cell in range
  grad_compute<T>(a, ic, in, sStage[threadIdx.x >> 6], g);
}

// Gradient and the fluxes of the chunk's own faces in one launch (gather
// mode, whole-mesh launches over the mesh order, forward Euler level steps).
// Block b takes cells [256 b, 256 b + 256) (a chunk), stages their face
// values in LDS as k_grad does, and stores only the half-faces whose other
// cell lies outside the chunk (to the compact array); after a barrier it
// computes the active faces with both sides in the chunk (and its boundary
// faces) from the staged values and stores their fluxes.  Their face values
// never leave the chip, and the flux kernel is left with the faces between
// chunks.  FEAT = 2: the learned guess, the network evaluated once per wave
// and pass over the chunk's faces as in k_flux_feat.  The face values,
// fluxes and counters are those of k_grad followed by the flux kernel, bit
// for bit.
template <typename T, bool G14, int FEAT>
__global__ __launch_bounds__(kBlock) void k_grad_flux(GradArgs<T> g, FluxArgs<T> f,
                                                      LocalFaces lf,
                                                      const uint32_t* __restrict__ fpack,
                                                      int tau_s) {
  __shared__ T sStage[kBlock / 64][kStageVals];
  __shared__ __attribute__((aligned(16))) uint16_t sNet[FEAT ? (kBlock / 64) * kMlpFwdLds : 8];
  const int chunk = xcd_block();
  const int idx = chunk * kBlock + threadIdx.x;
  // every wave reaches the barrier below: a lane past the end or outside the
  // key range computes its copy of a cell and stores nothing
  const int ic = idx < g.count ? idx : g.count - 1;
  const GradIn<T> gi = grad_load<T>(g, ic);
  const bool in = idx < g.count && g.key[idx] <= g.key_max;
  // the face values of the slots across chunks go to the compact array, the
  // others stay in LDS
  if (__ballot(in) != 0ull) grad_compute<T>(g, ic, in, sStage[threadIdx.x >> 6], gi, 0u);
  __syncthreads();
  // an active face has both cells in range (tau_g <= tau_f <= tau_s), so
  // both staged values are its face values
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  const double dt_min = flux_dt_min(f);
  const int q0 = lf.start[chunk], q1 = lf.start[chunk + 1];
  // the block's passes over its faces: the same count for every wave (the
  // network pass needs whole waves)
  for (int base = q0; base < q1; base += kBlock) {
    const int q = base + threadIdx.x;
    bool valid = q < q1;
    int2 e = make_int2(0, 0);
    int tf = 0;
    if (valid) {
      e = lf.face[q];
      // (the packed word of the face's first cell: its tau_f per face slot)
      tf = (int)((fpack[chunk * kBlock + (e.y & 255)] >> (4 * ((e.y >> 8) & 3))) & 15u);
      valid = tf <= tau_s;
    }
    if (FEAT == 0 && !valid) continue;
    const int lL = e.y & 255, sL = (e.y >> 8) & 3, lR = (e.y >> 10) & 255, sR = (e.y >> 18) & 3;
    const bool bnd = (e.y >> 20) & 1;
    T wl[5] = {1, 0, 0, 0, 1}, wr[5] = {1, 0, 0, 0, 1};
    if (valid) {
      const T* pl = &sStage[lL >> 6][sL * 320 + 5 * (lL & 63)];
      const T* pr = &sStage[lR >> 6][sR * 320 + 5 * (lR & 63)];
      for (int k = 0; k < 5; ++k) wl[k] = pl[k];
      for (int k = 0; k < 5; ++k) wr[k] = bnd ? wl[k] : pr[k];
    }
    const int4 r = make_int4(e.x, 0, bnd ? -1 : 0, tf);
    if (FEAT == 0) {
      T phi[5];
      SolveInfo one{0, 0, 0, 0, 0, 0, 0, 0};
      face_flux_w<T, G14>(f, e.x, !bnd, wl, wr, phi, one);
      add_info(info, one);
      store_face_flux(f, r, dt_min, phi, bnd && f.s.boundary == TAFV_BC_WALL, i0, i1, i2);
    } else {
      flux_feat_w<T, FEAT>(f, valid, r, wl, wr, dt_min, sNet + (threadIdx.x >> 6) * kMlpFwdLds,
                           info, i0, i1, i2);
    }
  }
  flush_counters(info, i0, i1, i2, f.dcount, f.dimpulse);
}

// ---------------------------------------------------------------------------
// face flux

// Colour scatter: the faces of one colour share no cell, so each thread
// reads, updates and writes both cells' accumulators with plain memory
// operations.  The accumulators are loaded before the flux is computed so
// their latency overlaps the solve.
template <int ORDER, typename T, bool G14>
__global__ __launch_bounds__(kBlock) void k_flux_colour(FluxArgs<T> a) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
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
// MOVE: through faces moving with their nodes (ALE form, see face_flux)
template <int ORDER, typename T, bool G14, bool MOVE = false>
__global__ __launch_bounds__(kBlock) void k_flux_store(FluxArgs<T> a) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  int4 r;
  if (flux_item(a, idx, r))
    flux_store_item<ORDER, T, G14, MOVE>(a, r, flux_dt_min(a), info, i0, i1, i2,
                                         flux_compact(a, idx));
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

// gamma = 1.4 flux with the optional features (statistics and face logging,
// learned guess)
template <int ORDER, typename T, int FEAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kFeatWaves<T>)))
void k_flux_feat(FluxArgs<T> a) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[(FEAT & 2) ? (kBlock / 64) * kMlpFwdLds : 8];
  int idx = xcd_block() * kBlock + threadIdx.x;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  int4 r;
  const bool valid = flux_item(a, idx, r);
  flux_feat_item<ORDER, T, FEAT>(a, valid, r, flux_dt_min(a), lds + (threadIdx.x >> 6) * kMlpFwdLds,
                                 info, i0, i1, i2, flux_compact(a, idx));
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cell_gather(int count, const int* __restrict__ list,
                                                        ListRanges rg,
                                                        int nc, const uint32_t* __restrict__ fpack,
                                                        const int* __restrict__ c2f,
                                                        const T* __restrict__ Q, double dt_min,
                                                        const double* __restrict__ vol,
                                                        double* __restrict__ U,
                                                        double* __restrict__ R, int tau_s,
                                                        int tau_upd, unsigned long long* dscal,
                                                        int dt_min_on_device, int first) {
  // first: a whole-mesh launch over the cells [first, count)
  int idx = first + xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  // dt_min_on_device: a launch enqueued before the host read dt_min back
  if (dt_min_on_device) dt_min = __longlong_as_double((long long)dscal[0]);
  if (!cell_gather_item<T>(range_cell(list, rg, idx), nc, fpack, c2f, Q, dt_min, vol, U, R,
                           tau_s, tau_upd))
    atomicOr(&dscal[2], 1ull);
}

// moving mesh: the same with the swept volumes and the cell volumes
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cell_gather_move(
    int count, const int* __restrict__ list, ListRanges rg, int nc,
    const uint32_t* __restrict__ fpack, const int* __restrict__ c2f, const T* __restrict__ Q,
    double dt_min, double* __restrict__ vol, double* __restrict__ U, double* __restrict__ R,
    int tau_s,
    int tau_upd, const double* __restrict__ sF, double* __restrict__ Rv,
    unsigned long long* dscal) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  if (!cell_gather_item<T, true>(range_cell(list, rg, idx), nc, fpack, c2f, Q, dt_min, vol, U,
                                 R, tau_s, tau_upd, sF, Rv, vol))
    atomicOr(&dscal[2], 1ull);
}


// moving mesh: each face moves with the mean velocity of its three nodes and
// sweeps volume at the rate sF = w_f . A_f (node velocities [n_nodes][3])
__global__ void k_face_speed(int nf, const int* __restrict__ fnode, const double* __restrict__ fA,
                             const double* __restrict__ vel, double* __restrict__ sF) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double* va = vel + 3 * (size_t)fnode[f];
  const double* vb = vel + 3 * (size_t)fnode[nf + f];
  const double* vc = vel + 3 * (size_t)fnode[2 * (size_t)nf + f];
  double w0 = (va[0] + vb[0] + vc[0]) / 3.0;
  double w1 = (va[1] + vb[1] + vc[1]) / 3.0;
  double w2 = (va[2] + vb[2] + vc[2]) / 3.0;
  sF[f] = w0 * fA[f] + w1 * fA[nf + f] + w2 * fA[2 * (size_t)nf + f];
}

// predictor/corrector form: predictions of the starting cells and the
// states at the end of the subiteration of the cells the next face passes
// read (nkey <= upd)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_predict(int nc, const uint32_t* __restrict__ fpack,
                                                    const int* __restrict__ c2f,
                                                    const T* __restrict__ Q0, double dt_min,
                                                    const double* __restrict__ vol,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ D,
                                                    double* __restrict__ Ut, int tau_s, int s,
                                                    const int8_t* __restrict__ nkey, int upd) {
  int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= nc) return;
  predict_item<T>(i, nc, fpack, c2f, Q0, dt_min, vol, U, D, Ut, tau_s, s, nkey, upd);
}

// predictor/corrector form: nkey = the smallest tau_g (ckey) over the cell
// and its face neighbours
__global__ __launch_bounds__(kBlock) void k_ring_keys(int nc, const int* __restrict__ nb,
                                                      const int8_t* __restrict__ ckey,
                                                      int8_t* __restrict__ nkey) {
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= nc) return;
  int n[4];
  for (int m = 0; m < 4; ++m) n[m] = nb[(size_t)m * nc + i];
  int k = ckey[i];
  for (int m = 0; m < 4; ++m)
    if (n[m] >= 0) k = min(k, (int)ckey[n[m]]);
  nkey[i] = (int8_t)k;
}

// predictor/corrector form: corrector sums of the listed cells
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cell_gather2(
    int count, const int* __restrict__ list, int n1, int off2, int nc,
    const uint32_t* __restrict__ fpack, const int* __restrict__ c2f, const T* __restrict__ Q,
    double dt_min, const double* __restrict__ vol, double* __restrict__ U,
    double* __restrict__ Ut, double* __restrict__ R, int tau_upd,
    unsigned long long* dscal) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  if (!cell_gather2_item<T>(list_cell(list, n1, off2, idx), nc, fpack, c2f, Q, dt_min, vol, U,
                            Ut, R, tau_upd))
    atomicOr(&dscal[2], 1ull);
}


// ---------------------------------------------------------------------------
// cells whose level step ends: U += R / V, R = 0

__global__ __launch_bounds__(kBlock) void k_update(int count, const int* __restrict__ list,
                                                   int n1, int off2,
                                                   const int8_t* __restrict__ lev, int tau_upd,
                                                   const double* __restrict__ vol,
                                                   double* __restrict__ U, double* __restrict__ R,
                                                   unsigned long long* dscal) {
  int idx = xcd_block() * kBlock + threadIdx.x;
  if (idx >= count) return;
  int i = list_cell(list, n1, off2, idx);
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

hipError_t launch_state_init_rows(hipStream_t s, int n, const int* perm, const double* d_prim,
                                  double gamma, double* U, double* R) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_init, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, perm, d_prim,
                     gamma - 1.0, U, R);
  return hipGetLastError();
}

hipError_t launch_state_init(hipStream_t s, DevMesh& m, const double* d_prim, double gamma) {
  return launch_state_init_rows(s, m.nc, m.perm, d_prim, gamma, m.U, m.R);
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
                     m.c2f, m.fA, a.gas.g, a.cfl, m.dt, m.dscal, m.dmin,
                     m.moving ? m.sF : nullptr);
  hipLaunchKernelGGL(k_min_slots, dim3(1), dim3(64), 0, s, m.dmin, m.dscal, m.sweepf, m.chist);
  return hipGetLastError();
}

hipError_t launch_classify(hipStream_t s, DevMesh& m, const StepArgs& a) {
  hipLaunchKernelGGL(k_classify_sweep, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.dt,
                     m.dscal, a.level_margin, m.max_levels, m.nb_, m.lev, m.sweepf);
  // the classification took the first of the L - 1 sweeps
  for (int k = 1; k < m.max_levels - 1; ++k)
    hipLaunchKernelGGL(k_sweep_inplace, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.nb_,
                       m.lev, m.sweepf, k);
  return hipGetLastError();
}

// Keys, counts, scans and scatters of the face list and the cell lists; the
// cell scatter's first block then packs the host readback buffer m.rb.
hipError_t launch_partitions(hipStream_t s, DevMesh& m, int early_order) {
  static_assert(kMaxLevels + kCellKeys <= kMaxKeys, "the two cell lists share one scan");
  static_assert(kPartChunk == kBlock, "the key kernels count one block of items each");
  const int use_colour = m.scatter == TAFV_SCATTER_COLOUR;
  const int Kf = face_list_keys(m);
  const int Kc = early_order ? kMaxLevels + kCellKeys : kMaxLevels;
  const int nbf = partition_blocks(m.nf), nbc = partition_blocks(m.nc);
  hipLaunchKernelGGL(k_keys, dim3(nbf + nbc), dim3(kBlock), 0, s, m.nf, nbf, m.fhL, m.fhR,
                     m.fcol, use_colour, m.split_local ? m.flocal : nullptr, Kf, m.fkey,
                     m.pf.counts, m.nc, nbc, m.nb_, m.lev,
                     m.ckey, m.fpack, m.chist, early_order ? 0 : 1, m.pc.counts);
  if (early_order)
    hipLaunchKernelGGL(k_cell_list_keys, dim3(nbc), dim3(kBlock), 0, s, m.nc, nbc, m.nb_, m.lev,
                       m.ckey, m.fpack, m.lkey, early_order, m.pc.counts);
  if (m.nkey)
    hipLaunchKernelGGL(k_ring_keys, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc, m.nb_,
                       m.ckey, m.nkey);
  hipLaunchKernelGGL(k_part_scan, dim3(Kf + Kc), dim3(kScanThreads), 0, s, Kf, nbf, m.pf.counts,
                     m.pf.offs, m.pf.tot, nbc, m.pc.counts, m.pc.offs, m.pc.tot);
  const Readback none{nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  hipLaunchKernelGGL((k_part_scatter<ByteKey, FaceWriter, IndexWriter>), dim3(nbf), dim3(64), 0,
                     s, m.nf, ByteKey{m.fkey}, Kf, FaceWriter{m.frec, m.split_local ? m.fxL : m.fhL, m.split_local ? m.fxR : m.fhR}, m.pf.start,
                     ByteKey{nullptr}, 0, IndexWriter{nullptr}, nullptr, nbf, m.pf.offs,
                     m.pf.tot, none);
  const Readback rb{m.dscal, m.pf.start, Kf, m.pc.start, early_order ? m.pg.start : nullptr,
                    m.chist, m.rb};
  if (early_order)
    hipLaunchKernelGGL((k_part_scatter<ByteKey, IndexWriter, IndexWriter>), dim3(nbc), dim3(64),
                       0, s, m.nc, ByteKey{m.ckey}, kMaxLevels, IndexWriter{m.pc.list},
                       m.pc.start, ByteKey{m.lkey}, kCellKeys, IndexWriter{m.pg.list},
                       m.pg.start, nbc, m.pc.offs, m.pc.tot, rb);
  else  // the gather's list serves time order 1 only
    hipLaunchKernelGGL((k_part_scatter<ByteKey, IndexWriter, IndexWriter>), dim3(nbc), dim3(64),
                       0, s, m.nc, ByteKey{m.ckey}, kMaxLevels, IndexWriter{m.pc.list},
                       m.pc.start, ByteKey{nullptr}, 0, IndexWriter{nullptr}, nullptr, nbc,
                       m.pc.offs, m.pc.tot, rb);
  return hipGetLastError();
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
hipError_t launch_rows_to_caller_f64(hipStream_t s, int n, const int* perm, const double* src,
                                    double* dst) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rows_to_caller<double>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, 5,
                     perm, src, dst);
  return hipGetLastError();
}
hipError_t launch_rows_to_caller_i8(hipStream_t s, int n, const int* perm, const int8_t* src,
                                   int8_t* dst) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rows_to_caller<int8_t>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, 1,
                     perm, src, dst);
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

// A launch that covers most of the mesh visits it in its own order (a
// whole-mesh launch) rather than through a level-sorted list: neighbours are
// then close in time, and their states and shared face fluxes are still in
// L2 when read again.
static bool whole_mesh(int64_t count, int64_t nc) { return count * 100 >= kWholeMeshPct * nc; }
bool grad_whole_mesh(const DevMesh& m, int64_t count) { return whole_mesh(count, m.nc); }
bool faces_whole_mesh(const DevMesh& m, int64_t count) { return whole_mesh(count, m.nf); }

hipError_t launch_grad(hipStream_t s, DevMesh& m, const StepArgs& a, CellRange r, int tau_g,
                       const double* U) {
  int count = r.count();
  if (count <= 0) return hipSuccess;
  if (!U) U = m.U;
  const int* list = m.pc.list;
  if (r.n2 == 0 && whole_mesh(count, m.nc)) {  // the cells of tau_g <= tau_g, in mesh order
    list = nullptr;
    count = m.nc;
  }
  const int* xb = m.split_local ? m.xb : nullptr;
  if (a.precision == TAFV_FP32_FLUX) {
    GradArgs<float> g{list, count, m.nc, m.nf, U, m.nb_, m.grc32, m.fA,
                      (float*)m.Wf, a.gas.gm1, a.boundary, m.moving ? m.sF : nullptr,
                      r.n1, r.off2, m.ckey, tau_g, xb ? (float*)m.Wx : nullptr, xb};
    hipLaunchKernelGGL(k_grad<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s, g);
  } else {
    GradArgs<double> g{list, count, m.nc, m.nf, U, m.nb_, m.grc, m.fA,
                       (double*)m.Wf, a.gas.gm1, a.boundary, m.moving ? m.sF : nullptr,
                       r.n1, r.off2, m.ckey, tau_g, xb ? (double*)m.Wx : nullptr, xb};
    hipLaunchKernelGGL(k_grad<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s, g);
  }
  return hipGetLastError();
}

template <typename T>
static void grad_flux_launch(hipStream_t s, const DevMesh& m, const GradArgs<T>& g,
                             const FluxArgs<T>& f, int feat, bool is14, int tau_s) {
  const LocalFaces lf{m.lf_start, m.lf_face};
  const dim3 grid(blocks_for(m.nc)), block(kBlock);
  if (feat == 2)
    hipLaunchKernelGGL((k_grad_flux<T, true, 2>), grid, block, 0, s, g, f, lf, m.fpack, tau_s);
  else if (is14)
    hipLaunchKernelGGL((k_grad_flux<T, true, 0>), grid, block, 0, s, g, f, lf, m.fpack, tau_s);
  else
    hipLaunchKernelGGL((k_grad_flux<T, false, 0>), grid, block, 0, s, g, f, lf, m.fpack, tau_s);
}

hipError_t launch_grad_flux(hipStream_t s, DevMesh& m, const StepArgs& a, int tau_s,
                            const FluxFeatures& ft, bool dt_min_on_device) {
  static_assert(kFuseChunk == kBlock && kChunkCells == kBlock, "a chunk is one block of cells");
  if (m.nc <= 0) return hipSuccess;
  // the learned guess alone (FEAT 2, gamma 1.4), or no features
  if (ft.feat != 0 && (ft.feat != 2 || !a.gas.is14)) return hipErrorInvalidValue;
  if (!m.split_local) return hipErrorInvalidValue;
  const unsigned long long* dtd = dt_min_on_device ? m.dscal : nullptr;
  if (a.precision == TAFV_FP32_FLUX) {
    GradArgs<float> g{nullptr, m.nc, m.nc, m.nf, m.U, m.nb_, m.grc32, m.fA, (float*)m.Wf,
                      a.gas.gm1, a.boundary, nullptr, 0, 0, m.ckey, tau_s, (float*)m.Wx, m.xb};
    FluxArgs<float> f{m.frec, 0, m.nf, m.nc, m.fA32, m.U, (const float*)m.Wf, m.R, (float*)m.Q,
                      m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                      ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                      0, nullptr, nullptr, dtd};
    grad_flux_launch<float>(s, m, g, f, ft.feat, a.gas.is14, tau_s);
  } else {
    GradArgs<double> g{nullptr, m.nc, m.nc, m.nf, m.U, m.nb_, m.grc, m.fA, (double*)m.Wf,
                       a.gas.gm1, a.boundary, nullptr, 0, 0, m.ckey, tau_s, (double*)m.Wx,
                       m.xb};
    FluxArgs<double> f{m.frec, 0, m.nf, m.nc, m.fA, m.U, (const double*)m.Wf, m.R, (double*)m.Q,
                       m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                       ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                       0, nullptr, nullptr, dtd};
    grad_flux_launch<double>(s, m, g, f, ft.feat, a.gas.is14, tau_s);
  }
  return hipGetLastError();
}

template <typename T, bool G14>
static void flux_launch(hipStream_t s, int order, int scatter, int count, const FluxArgs<T>& f) {
  dim3 g(blocks_for(count)), b(kBlock);
  if (f.sF) {  // moving mesh (gather mode)
    if (order == 2) hipLaunchKernelGGL((k_flux_store<2, T, G14, true>), g, b, 0, s, f);
    else hipLaunchKernelGGL((k_flux_store<1, T, G14, true>), g, b, 0, s, f);
    return;
  }
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
                       const FluxFeatures& ft, const double* U, void* Q, int pass_mode,
                       const void* Qpred, bool dt_min_on_device, int first2, int count2,
                       int key_max) {
  // with the chunk-local faces kept apart, the first range holds faces
  // between chunks, whose records point into the compact face values
  const bool compact1 = m.split_local && count > 0;
  // most faces active: walk all faces in face order instead of the list
  const bool face_order = key_max >= 0 && !m.split_local && first == 0 && count2 <= 0 &&
                          m.scatter == TAFV_SCATTER_GATHER && whole_mesh(count, m.nf);
  if (count <= 0) {  // the second range alone
    first = first2;
    count = count2;
    count2 = 0;
  }
  if (count + count2 <= 0) return hipSuccess;
  const int n1 = count, off2 = first2 - first;
  count += count2;
  const int4* rec = m.frec + first;
  if (!U) U = m.U;
  if (!Q) Q = m.Q;
  if (a.precision == TAFV_FP32_FLUX) {
    FluxArgs<float> f{rec, count, m.nf, m.nc, m.fA32, U, (const float*)m.Wf, m.R, (float*)Q, m.dcount,
                      m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                      ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                      pass_mode, (const float*)Qpred, m.moving ? m.sF : nullptr,
                      dt_min_on_device ? m.dscal : nullptr, n1, off2,
                      compact1 ? (const float*)m.Wx : nullptr,
                      (ft.feat & 1) ? m.dnewton : nullptr};
    if (face_order) {
      f.count = count = m.nf;
      f.fkey = m.fkey;
      f.key_max = key_max;
      f.fhL = m.fhL;
      f.fhR = m.fhR;
    }
    if (ft.feat && a.gas.is14 && m.scatter == TAFV_SCATTER_GATHER && !m.moving)
      flux_feat_launch<float>(s, a.order, ft.feat, count, f);
    else if (a.gas.is14) flux_launch<float, true>(s, a.order, m.scatter, count, f);
    else flux_launch<float, false>(s, a.order, m.scatter, count, f);
  } else {
    FluxArgs<double> f{rec, count, m.nf, m.nc, m.fA, U, (const double*)m.Wf, m.R, (double*)Q,
                       m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                       ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                       pass_mode, (const double*)Qpred, m.moving ? m.sF : nullptr,
                       dt_min_on_device ? m.dscal : nullptr, n1, off2,
                       compact1 ? (const double*)m.Wx : nullptr,
                       (ft.feat & 1) ? m.dnewton : nullptr};
    if (face_order) {
      f.count = count = m.nf;
      f.fkey = m.fkey;
      f.key_max = key_max;
      f.fhL = m.fhL;
      f.fhR = m.fhR;
    }
    if (ft.feat && a.gas.is14 && m.scatter == TAFV_SCATTER_GATHER && !m.moving)
      flux_feat_launch<double>(s, a.order, ft.feat, count, f);
    else if (a.gas.is14) flux_launch<double, true>(s, a.order, m.scatter, count, f);
    else flux_launch<double, false>(s, a.order, m.scatter, count, f);
  }
  return hipGetLastError();
}

hipError_t launch_cell_gather(hipStream_t s, DevMesh& m, const ListRanges& r, int tau_s,
                              int tau_upd, double dt_min, int precision, bool dt_min_on_device) {
  int count = r.count();
  if (count <= 0) return hipSuccess;
  // a whole-mesh launch: the cells outside the ranges find nothing to do
  const int* list = m.pg.list;
  if (whole_mesh(count, m.nc)) {
    list = nullptr;
    count = m.nc;
  }
  if (m.moving) {
    if (precision == TAFV_FP32_FLUX)
      hipLaunchKernelGGL(k_cell_gather_move<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s,
                         count, list, r, m.nc, m.fpack, m.c2f,
                         (const float*)m.Q, dt_min, m.vol, m.U, m.R, tau_s, tau_upd, m.sF, m.Rv,
                         m.dscal);
    else
      hipLaunchKernelGGL(k_cell_gather_move<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s,
                         count, list, r, m.nc, m.fpack, m.c2f,
                         (const double*)m.Q, dt_min, m.vol, m.U, m.R, tau_s, tau_upd, m.sF, m.Rv,
                         m.dscal);
    return hipGetLastError();
  }
  if (precision == TAFV_FP32_FLUX)
    hipLaunchKernelGGL(k_cell_gather<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s, count,
                       list, r, m.nc, m.fpack, m.c2f, (const float*)m.Q, dt_min,
                       m.vol, m.U, m.R, tau_s, tau_upd, m.dscal, dt_min_on_device ? 1 : 0, 0);
  else
    hipLaunchKernelGGL(k_cell_gather<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s, count,
                       list, r, m.nc, m.fpack, m.c2f, (const double*)m.Q, dt_min,
                       m.vol, m.U, m.R, tau_s, tau_upd, m.dscal, dt_min_on_device ? 1 : 0, 0);
  return hipGetLastError();
}

// One stage of a pipelined whole-mesh subiteration: the gradients of the
// cells [c0, c1) of tau_g <= tau_s, or the fluxes of the faces [f0, f1) of
// tau_f <= tau_s in face order, or the gather of the cells [c0, c1).
hipError_t launch_grad_chunk(hipStream_t s, DevMesh& m, const StepArgs& a, int tau_s, int c0,
                             int c1) {
  if (c1 <= c0) return hipSuccess;
  const dim3 grid(blocks_for(c1 - c0)), block(kBlock);
  if (a.precision == TAFV_FP32_FLUX) {
    GradArgs<float> g{nullptr, c1, m.nc, m.nf, m.U, m.nb_, m.grc32, m.fA, (float*)m.Wf,
                      a.gas.gm1, a.boundary, nullptr, 0, 0, m.ckey, tau_s};
    g.first = c0;
    hipLaunchKernelGGL(k_grad<float>, grid, block, 0, s, g);
  } else {
    GradArgs<double> g{nullptr, c1, m.nc, m.nf, m.U, m.nb_, m.grc, m.fA, (double*)m.Wf,
                       a.gas.gm1, a.boundary, nullptr, 0, 0, m.ckey, tau_s};
    g.first = c0;
    hipLaunchKernelGGL(k_grad<double>, grid, block, 0, s, g);
  }
  return hipGetLastError();
}

hipError_t launch_flux_chunk(hipStream_t s, DevMesh& m, const StepArgs& a,
                             const FluxFeatures& ft, int tau_s, int f0, int f1,
                             bool dt_min_on_device) {
  if (f1 <= f0) return hipSuccess;
  const int n = f1 - f0;
  const unsigned long long* dtd = dt_min_on_device ? m.dscal : nullptr;
  if (a.precision == TAFV_FP32_FLUX) {
    FluxArgs<float> f{m.frec, f1, m.nf, m.nc, m.fA32, m.U, (const float*)m.Wf, m.R, (float*)m.Q,
                      m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                      ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                      0, nullptr, nullptr, dtd};
    f.dnewton = (ft.feat & 1) ? m.dnewton : nullptr;
    f.fkey = m.fkey;
    f.key_max = tau_s;
    f.fhL = m.fhL;
    f.fhR = m.fhR;
    f.ffirst = f0;
    if (ft.feat && a.gas.is14) flux_feat_launch<float>(s, a.order, ft.feat, n, f);
    else if (a.gas.is14) flux_launch<float, true>(s, a.order, m.scatter, n, f);
    else flux_launch<float, false>(s, a.order, m.scatter, n, f);
  } else {
    FluxArgs<double> f{m.frec, f1, m.nf, m.nc, m.fA, m.U, (const double*)m.Wf, m.R, (double*)m.Q,
                       m.dcount, m.dimpulse, a, ft.mlp, ft.log_rows, ft.log_count, ft.log_cap,
                       ft.log_rate, ft.log_seed, ft.subit, ft.guess_gate, ft.guess_strength,
                       0, nullptr, nullptr, dtd};
    f.dnewton = (ft.feat & 1) ? m.dnewton : nullptr;
    f.fkey = m.fkey;
    f.key_max = tau_s;
    f.fhL = m.fhL;
    f.fhR = m.fhR;
    f.ffirst = f0;
    if (ft.feat && a.gas.is14) flux_feat_launch<double>(s, a.order, ft.feat, n, f);
    else if (a.gas.is14) flux_launch<double, true>(s, a.order, m.scatter, n, f);
    else flux_launch<double, false>(s, a.order, m.scatter, n, f);
  }
  return hipGetLastError();
}

hipError_t launch_gather_chunk(hipStream_t s, DevMesh& m, int tau_s, int tau_upd, double dt_min,
                               int precision, int c0, int c1, bool dt_min_on_device) {
  if (c1 <= c0) return hipSuccess;
  const ListRanges none{};
  const dim3 grid(blocks_for(c1 - c0)), block(kBlock);
  if (precision == TAFV_FP32_FLUX)
    hipLaunchKernelGGL(k_cell_gather<float>, grid, block, 0, s, c1, (const int*)nullptr, none, m.nc,
                       m.fpack,
                       m.c2f, (const float*)m.Q, dt_min, m.vol, m.U, m.R, tau_s, tau_upd,
                       m.dscal, dt_min_on_device ? 1 : 0, c0);
  else
    hipLaunchKernelGGL(k_cell_gather<double>, grid, block, 0, s, c1, (const int*)nullptr, none,
                       m.nc, m.fpack, m.c2f, (const double*)m.Q, dt_min, m.vol, m.U, m.R, tau_s,
                       tau_upd, m.dscal, dt_min_on_device ? 1 : 0, c0);
  return hipGetLastError();
}

hipError_t launch_predict(hipStream_t s, DevMesh& m, int tau_s, int sub, int upd,
                          double dt_min, int precision) {
  if (m.nc <= 0) return hipSuccess;
  if (!m.nkey) return hipErrorInvalidValue;
  if (precision == TAFV_FP32_FLUX)
    hipLaunchKernelGGL(k_predict<float>, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc,
                       m.fpack, m.c2f, (const float*)m.Q0, dt_min, m.vol, m.U, m.D, m.Ut,
                       tau_s, sub, m.nkey, upd);
  else
    hipLaunchKernelGGL(k_predict<double>, dim3(blocks_for(m.nc)), dim3(kBlock), 0, s, m.nc,
                       m.fpack, m.c2f, (const double*)m.Q0, dt_min, m.vol, m.U, m.D, m.Ut,
                       tau_s, sub, m.nkey, upd);
  return hipGetLastError();
}

hipError_t launch_cell_gather2(hipStream_t s, DevMesh& m, CellRange r, int tau_upd,
                               double dt_min, int precision) {
  const int count = r.count();
  if (count <= 0) return hipSuccess;
  if (precision == TAFV_FP32_FLUX)
    hipLaunchKernelGGL(k_cell_gather2<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s,
                       count, m.pc.list, r.n1, r.off2, m.nc, m.fpack, m.c2f, (const float*)m.Q,
                       dt_min, m.vol, m.U, m.Ut, m.R, tau_upd, m.dscal);
  else
    hipLaunchKernelGGL(k_cell_gather2<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s,
                       count, m.pc.list, r.n1, r.off2, m.nc, m.fpack, m.c2f, (const double*)m.Q,
                       dt_min, m.vol, m.U, m.Ut, m.R, tau_upd, m.dscal);
  return hipGetLastError();
}

hipError_t launch_face_speed(hipStream_t s, DevMesh& m, const double* d_vel) {
  if (m.nf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_speed, dim3(blocks_for(m.nf)), dim3(kBlock), 0, s, m.nf, m.fnode,
                     m.fA, d_vel, m.sF);
  return hipGetLastError();
}

hipError_t launch_vol_to_caller(hipStream_t s, DevMesh& m, const double* src, double* dst) {
  return rows_to_caller<double>(s, m, 1, src, dst);
}

hipError_t launch_update(hipStream_t s, DevMesh& m, CellRange r, int tau_upd) {
  const int count = r.count();
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(blocks_for(count)), dim3(kBlock), 0, s, count, m.pc.list,
                     r.n1, r.off2, m.lev, tau_upd, m.vol, m.U, m.R, m.dscal);
  return hipGetLastError();
}

}  // namespace tafv
