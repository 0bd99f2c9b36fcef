// Batched form: many independent tetrahedral meshes, each with its own
// temporal levels and schedule (Sec. 2.2, Alg. 2), advanced together.
//
// The meshes are merged into one set of device arrays (cell, face and
// half-face ids offset per mesh, every face and cell of a mesh in one
// contiguous segment).  Each mesh's schedule (level cap, theta, phase,
// dt_min, list starts, active counts) lives in a device table, so a
// subiteration is a fixed sequence of launches that a HIP graph can hold:
//   k_b_begin       meshes at an iteration start are marked to reclassify;
//   k_b_dt ... keys time step, per-mesh dt_min, levels, neighbour sweeps,
//                   keys and per-mesh stable partitions by level (only the
//                   marked meshes do work);
//   k_b_sched       one block: theta, the subiteration level tau_s, the
//                   levels whose steps end, active counts and the tile
//                   prefix of each work class over all meshes;
//   k_b_grad / k_b_flux* / k_b_gather
//                   persistent kernels over the active prefixes of all
//                   meshes, taken as one list of 256-item tiles.
// The per-item arithmetic is the single-mesh path's (kernels_dev.h), so a
// mesh advanced in a batch gets the same bits as on its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.h"
#include "kernels_dev.h"
#include "mlp.h"
#include "tafv_internal.h"

namespace tafv {
namespace {

constexpr int kChunk = 1024;        // partition chunk: 16 waves of 64
constexpr int kUnit = 64;           // work unit of the gradient, flux and cell kernels
constexpr int kStaticBlocksPerCU = 4;
// persistent grids of the reclassification kernels: more blocks than the
// work kernels take, as these do little arithmetic per memory trip (8 per
// CU measured faster than 4 and 16 on the 128-mesh workload)
constexpr int kReclassBlocksPerCU = 8;
constexpr int kGraphSpan = 32;      // subiterations per captured graph
constexpr int kMaxBatchMeshes = 8192;  // prefix arrays staged in LDS (32 KB)

// the mesh whose tiles hold tile t: tp[m] <= t < tp[m + 1] (tp[M] > t)
__device__ inline int find_mesh(const int32_t* __restrict__ tp, int M, int t) {
  int lo = 0, hi = M;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tp[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// the mesh of unit u >= u0 of a block whose first unit u0 lies in mesh m0:
// one search per block (every wave searches the same u0), then a short walk
__device__ inline int mesh_after(const int32_t* __restrict__ tp, int m0, int u) {
  int m = m0;
  while (u >= tp[m + 1]) ++m;
  return m;
}

// The grids here are sized before the work is known (persistent grids, or
// the static count of a work class), so often only part of a grid has work.
// The hardware hands blocks out in index order, round-robin over the 8 XCDs:
// the first n blocks are the ones that work, spread over all XCDs, each
// taking its XCD-remapped rank among those n (ranks over the whole grid
// would leave the working ranks unevenly spread over the XCDs, and the
// persistent loops' strides would not match the working blocks).
// Number of blocks that take part in a loop over `count` items run by nb
// blocks (the grid, or one of its two halves, see split_half):
__device__ inline int loop_blocks(int count, int nb) { return min(nb, count); }
__device__ inline int loop_blocks(int count) { return loop_blocks(count, (int)gridDim.x); }
// The rank among them of block b of those nb, or `count` for a block that
// does not take part:
__device__ inline int loop_rank(int count, int b, int nb) {
  const int n = loop_blocks(count, nb);
  return b < n ? xcd_rank(b, n) : count;
}
__device__ inline int loop_rank(int count) {
  return loop_rank(count, (int)blockIdx.x, (int)gridDim.x);
}

// Two independent loops in one launch (the face and the cell classes of a
// reclassification step): blocks [0, h) run the first, [h, gridDim.x) the
// second, h a multiple of 8 so that a block's XCD is its index within its
// half modulo 8.
__device__ inline int split_half() { return (int)(gridDim.x >> 4) << 3; }

// Tiles of a launch: with n blocks taking part, block rank r takes tiles
// [(k n + r) grab, (k n + r + 1) grab) for k = 0, 1, ...  Block-uniform.
#define TILE_LOOP(total, grab)                                                      \
  for (int n_ = loop_blocks(((total) + (grab) - 1) / (grab)),                        \
           base_ = loop_rank(((total) + (grab) - 1) / (grab)) * (grab);             \
       base_ < (total); base_ += n_ * (grab))                                        \
    for (int t = base_, tend_ = min(base_ + (grab), (total)); t < tend_; ++t)

// The prefix array of a launch (M + 1 ints) is staged in LDS, where the
// per-tile binary search over it costs little (dynamic shared memory of
// (M + 1) * 4 bytes at launch).
#define STAGE_PREFIX(gp)                                                           \
  extern __shared__ int32_t s_pre[];                                             \
  for (int k_ = threadIdx.x; k_ <= M; k_ += blockDim.x) s_pre[k_] = (gp)[k_];    \
  __syncthreads()

// ---- iteration start ----------------------------------------------------
// Meshes at an iteration start (phase 0) reclassify.  The tiles of the
// reclassification kernels cover those meshes only: rp[kind][M + 1] are
// prefix sums over the marked meshes of their static tile counts (kind 0
// cell tiles, 1 face tiles, 2 cell chunks, 3 face chunks).

__global__ __launch_bounds__(1024) void k_b_begin(BatchSched* S, int M, int reclassify,
                                                  const int32_t* __restrict__ ct,
                                                  const int32_t* __restrict__ ft,
                                                  const int32_t* __restrict__ cc,
                                                  const int32_t* __restrict__ fc,
                                                  int32_t* __restrict__ rp) {
  __shared__ int sh[4][1024];
  const int tid = threadIdx.x;
  const int32_t* st[4] = {ct, ft, cc, fc};
  int carry[4] = {0, 0, 0, 0};
  for (int b = 0; b < M; b += blockDim.x) {
    const int m = b + tid;
    int n[4] = {0, 0, 0, 0};
    if (m < M) {
      BatchSched& s = S[m];
      int rc = s.phase == 0 && (reclassify || !s.classified);
      s.reclass = rc;
      if (rc) {
        s.dtbits = 0x7ff0000000000000ull;  // +inf
        for (int k = 0; k < kMaxKeys; ++k) s.hist[k] = 0;
        for (int w = 0; w < 4; ++w) n[w] = st[w][m + 1] - st[w][m];
      }
    }
    for (int w = 0; w < 4; ++w) sh[w][tid] = n[w];
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int y[4];
      for (int w = 0; w < 4; ++w) y[w] = tid >= off ? sh[w][tid - off] : 0;
      __syncthreads();
      for (int w = 0; w < 4; ++w) sh[w][tid] += y[w];
      __syncthreads();
    }
    for (int w = 0; w < 4; ++w) {
      if (m < M) rp[w * (M + 1) + m] = carry[w] + sh[w][tid] - n[w];
      carry[w] += sh[w][1023];
    }
    __syncthreads();
  }
  if (tid < 4) rp[tid * (M + 1) + M] = carry[tid];
}

__global__ __launch_bounds__(kBlock) void k_b_dt(const int32_t* __restrict__ rp, BatchSched* S,
                                                 int M, int NC, int NF,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ vol,
                                                 const int* __restrict__ c2f,
                                                 const double* __restrict__ fA, double gamma,
                                                 double cfl, double* __restrict__ dt,
                                                 double* __restrict__ tmin,
                                                 unsigned long long* flag) {
  STAGE_PREFIX(rp);
  __shared__ double smin[kBlock / 64];
  const int total = s_pre[M];
  TILE_LOOP(total, 1) {
    int m = find_mesh(s_pre, M, t);
    int i = S[m].c0 + (t - s_pre[m]) * kBlock + threadIdx.x;
    double dti = INFINITY;
    if (i < S[m].c0 + S[m].nc) {
      bool bad = false;
      dti = dt_item(i, NC, NF, U, vol, c2f, fA, gamma, cfl, bad);
      if (bad) atomicOr(flag, 1ull);
      dt[i] = dti;
    }
    double v = wave_min(dti);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 1; k < kBlock / 64; ++k) v = fmin(v, smin[k]);
      tmin[t] = v;  // the tile's minimum; k_b_reduce takes the mesh's
    }
  }
}

// Per marked mesh (one block each): dt_min from its tiles' minima (tmin
// given) or the (tau_g, tau) histogram from its tiles' histograms (thist
// given), in place of per-tile atomics on the mesh's entry (which
// serialised on large meshes).
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_b_reduce(const int32_t* __restrict__ rp,
                                                             BatchSched* S, int M,
                                                             const double* __restrict__ tmin,
                                                             const int* __restrict__ thist) {
  constexpr int G = kReduceThreads / 64;  // groups of 64 bins
  __shared__ double sm[kReduceThreads];
  __shared__ int sh[G][kMaxKeys];
  const int m = blockIdx.x;
  if (m >= M || !S[m].reclass) return;
  const int t0 = rp[m], t1 = rp[m + 1], tid = threadIdx.x;
  if (tmin) {
    double v = INFINITY;
    for (int t = t0 + tid; t < t1; t += kReduceThreads) v = fmin(v, tmin[t]);
    sm[tid] = v;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
      if (tid < off) sm[tid] = fmin(sm[tid], sm[tid + off]);
      __syncthreads();
    }
    if (tid == 0) S[m].dtbits = (unsigned long long)__double_as_longlong(sm[0]);
  }
  if (thist) {
    // group g sums tiles t0 + g, t0 + g + G, ...; four loads in flight per
    // thread
    const int g = tid >> 6, k = tid & 63;
    int a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int t = t0 + g;
    for (; t + 3 * G < t1; t += 4 * G) {
      a0 += thist[(size_t)t * kMaxKeys + k];
      a1 += thist[(size_t)(t + G) * kMaxKeys + k];
      a2 += thist[(size_t)(t + 2 * G) * kMaxKeys + k];
      a3 += thist[(size_t)(t + 3 * G) * kMaxKeys + k];
    }
    for (; t < t1; t += G) a0 += thist[(size_t)t * kMaxKeys + k];
    sh[g][k] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (tid < kMaxKeys) {
      int sum = 0;
      for (int q = 0; q < G; ++q) sum += sh[q][tid];
      S[m].hist[tid] = sum;
    }
  }
}

// levels from each mesh's dt ratio together with the first lowering sweep
// (a neighbour's level is classified from its own time step)
__global__ __launch_bounds__(kBlock) void k_b_classify(const int32_t* __restrict__ rp,
                                                       const BatchSched* S, int M, int NC,
                                                       const double* __restrict__ dt,
                                                       double margin,
                                                       const int* __restrict__ nb,
                                                       int8_t* __restrict__ lev) {
  STAGE_PREFIX(rp);
  const int total = s_pre[M];
  TILE_LOOP(total, 1) {
    int m = find_mesh(s_pre, M, t);
    int i = S[m].c0 + (t - s_pre[m]) * kBlock + threadIdx.x;
    if (i < S[m].c0 + S[m].nc) {
      const double dtmin = __longlong_as_double((long long)S[m].dtbits);
      const int L = S[m].L;
      int n[4];
      double dn[4];
      for (int q = 0; q < 4; ++q) n[q] = nb[(size_t)q * NC + i];
      for (int q = 0; q < 4; ++q) dn[q] = dt[n[q] >= 0 ? n[q] : i];
      int tl = classify_item(dt[i], dtmin, margin, L);
      for (int q = 0; q < 4; ++q)
        if (n[q] >= 0) tl = min(tl, classify_item(dn[q], dtmin, margin, L) + 1);
      lev[i] = (int8_t)tl;
    }
  }
}

// lowering sweep k >= 1 in place for the meshes with k < L - 1 (a neighbour
// read while it is lowered gives its old or new level, both at or above the
// final one, so L - 1 sweeps reach the same levels as L - 1 Jacobi sweeps)
__global__ __launch_bounds__(kBlock) void k_b_sweep(const int32_t* __restrict__ rp,
                                                    const BatchSched* S, int M, int NC, int k,
                                                    const int* __restrict__ nb,
                                                    int8_t* lev) {
  STAGE_PREFIX(rp);
  const int total = s_pre[M];
  TILE_LOOP(total, 1) {
    int m = find_mesh(s_pre, M, t);
    if (k >= S[m].L - 1) continue;
    int i = S[m].c0 + (t - s_pre[m]) * kBlock + threadIdx.x;
    if (i < S[m].c0 + S[m].nc) lev[i] = sweep_item(i, NC, nb, lev);
  }
}

// Keys of the marked meshes after the sweeps, cells and faces in one
// launch (split_half): per cell tau_g, the packed face word and its tile's
// (tau_g, tau) histogram; per face tau_f.
__global__ __launch_bounds__(kBlock) void k_b_keys(const int32_t* __restrict__ rc,
                                                   const int32_t* __restrict__ rf,
                                                   BatchSched* S, int M, int NC,
                                                   const int* __restrict__ nb,
                                                   const int8_t* __restrict__ lev,
                                                   int8_t* __restrict__ ckey,
                                                   uint32_t* __restrict__ fpack,
                                                   int* __restrict__ thist,
                                                   const int* __restrict__ fhL,
                                                   const int* __restrict__ fhR,
                                                   int8_t* __restrict__ fkey) {
  const int h = split_half();
  const bool faces = (int)blockIdx.x >= h;  // block-uniform
  const int b = faces ? (int)blockIdx.x - h : (int)blockIdx.x;
  const int nbk = faces ? (int)gridDim.x - h : h;
  STAGE_PREFIX(faces ? rf : rc);
  __shared__ int hs[kMaxKeys];
  const int total = s_pre[M];
  for (int t = loop_rank(total, b, nbk), n_ = loop_blocks(total, nbk); t < total; t += n_) {
    int m = find_mesh(s_pre, M, t);
    if (faces) {
      int f = S[m].f0 + (t - s_pre[m]) * kBlock + threadIdx.x;
      if (f < S[m].f0 + S[m].nf) fkey[f] = face_key_item(f, fhL, fhR, nullptr, lev, 0);
      continue;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x) hs[k] = 0;
    __syncthreads();
    int i = S[m].c0 + (t - s_pre[m]) * kBlock + threadIdx.x;
    const bool in = i < S[m].c0 + S[m].nc;
    int bin = in ? cell_key_item(i, NC, nb, lev, ckey, fpack) : 0;
    wave_hist_add(hs, in, bin);
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxKeys; k += blockDim.x) thist[(size_t)t * kMaxKeys + k] = hs[k];
  }
}

// cells that apply their fluxes at their step's start (kEarlyBit)
__global__ __launch_bounds__(kBlock) void k_b_cell_early(const int32_t* __restrict__ rp,
                                                         BatchSched* S, int M, int NC,
                                                         const int* __restrict__ nb,
                                                         const int8_t* __restrict__ lev,
                                                         const int8_t* __restrict__ ckey,
                                                         uint32_t* __restrict__ fpack, int order) {
  STAGE_PREFIX(rp);
  const int total = s_pre[M];
  TILE_LOOP(total, 1) {
    int m = find_mesh(s_pre, M, t);
    int i = S[m].c0 + (t - s_pre[m]) * kBlock + threadIdx.x;
    if (i < S[m].c0 + S[m].nc) cell_early_item(i, NC, nb, lev, ckey, fpack, order);
  }
}

// ---- per-mesh stable partitions by level ----------------------------------
// Chunk j of mesh m covers segment items [j kChunk, (j + 1) kChunk); the
// count of key k in that chunk sits at 8 cp[m] + k nch + j (cp: the static
// chunk prefix, nch chunks in the mesh), so one exclusive scan per mesh,
// started at the segment's first position, gives every (key, chunk) its
// first slot in the merged list.  rp: the chunk prefix over the meshes that
// reclassify.

// Per chunk of the marked meshes' items, the counts of each key, faces and
// cells in one launch (split_half: faces in the first half).  pre is the
// staged chunk prefix of the block's class.
template <typename Key>
__device__ inline void count_chunks(const int32_t* pre, const int32_t* __restrict__ cp,
                                    const BatchSched* S, int M, int faces, Key key,
                                    int32_t* __restrict__ counts, int* cnt, int b, int nbk) {
  const int lane = threadIdx.x;
  const int total = pre[M];
  for (int t = loop_rank(total, b, nbk), n_ = loop_blocks(total, nbk); t < total; t += n_) {
    int m = find_mesh(pre, M, t);
    int j = t - pre[m], nch = cp[m + 1] - cp[m];
    int b0 = faces ? S[m].f0 : S[m].c0;
    int end = b0 + (faces ? S[m].nf : S[m].nc);
    __syncthreads();
    if (lane < kMaxLevels) cnt[lane] = 0;
    __syncthreads();
    int first = b0 + j * kChunk;
    for (int step = 0; step < kChunk / 64; ++step) {
      int i = first + step * 64 + lane;
      bool valid = i < end;
      int k_mine = valid ? key(i) : -1;
      unsigned long long pending = __ballot(valid);
      while (pending) {
        int leader = __ffsll(pending) - 1;
        int k = __shfl(k_mine, leader, 64);
        unsigned long long msk = __ballot(k_mine == k);
        if (lane == leader) cnt[k] += __popcll(msk);
        pending &= ~msk;
      }
    }
    __syncthreads();
    if (lane < kMaxLevels) counts[kMaxLevels * cp[m] + lane * nch + j] = cnt[lane];
  }
}

template <typename Key>
__global__ __launch_bounds__(64) void k_b_part_count(const int32_t* __restrict__ rpf,
                                                     const int32_t* __restrict__ rpc,
                                                     const int32_t* __restrict__ fcp,
                                                     const int32_t* __restrict__ ccp,
                                                     const BatchSched* S, int M, Key fkey,
                                                     Key ckey, int32_t* __restrict__ fcounts,
                                                     int32_t* __restrict__ ccounts) {
  const int h = split_half();
  const bool cells = (int)blockIdx.x >= h;  // block-uniform
  STAGE_PREFIX(cells ? rpc : rpf);
  __shared__ int cnt[kMaxLevels];
  if (cells)
    count_chunks(s_pre, ccp, S, M, 0, ckey, ccounts, cnt, (int)blockIdx.x - h,
                 (int)gridDim.x - h);
  else
    count_chunks(s_pre, fcp, S, M, 1, fkey, fcounts, cnt, (int)blockIdx.x, h);
}

// one block per mesh and class (blocks [0, M) the faces, [M, 2M) the
// cells): exclusive scan of its counts in place, plus the list starts per
// level
__global__ __launch_bounds__(256) void k_b_part_scan(const int32_t* __restrict__ fcp,
                                                     const int32_t* __restrict__ ccp,
                                                     BatchSched* S, int M,
                                                     int32_t* __restrict__ fcounts,
                                                     int32_t* __restrict__ ccounts) {
  __shared__ int sh[256];
  const int faces = (int)blockIdx.x < M;
  const int m = faces ? (int)blockIdx.x : (int)blockIdx.x - M;
  if (m >= M || !S[m].reclass) return;
  const int32_t* cp = faces ? fcp : ccp;
  int32_t* counts = faces ? fcounts : ccounts;
  const int tid = threadIdx.x;
  const int nch = cp[m + 1] - cp[m];
  const int n = kMaxLevels * nch;
  int32_t* c = counts + kMaxLevels * cp[m];
  const int b0 = faces ? S[m].f0 : S[m].c0;
  const int cnt_all = faces ? S[m].nf : S[m].nc;
  int carry = b0;
  for (int b = 0; b < n; b += 256) {
    int x = b + tid < n ? c[b + tid] : 0;
    sh[tid] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      int y = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += y;
      __syncthreads();
    }
    if (b + tid < n) c[b + tid] = carry + sh[tid] - x;
    int tot = sh[255];
    __syncthreads();
    carry += tot;
  }
  int32_t* start = faces ? S[m].fstart : S[m].cstart;
  if (tid < kMaxLevels) start[tid] = c[tid * nch];
  if (tid == 0) start[kMaxLevels] = b0 + cnt_all;
}

// The stable scatter of the marked meshes' items into their level-sorted
// lists, faces and cells in one launch (split_half: faces in the first
// half).  pre is the staged chunk prefix of the block's class.
template <typename Key, typename Writer>
__device__ inline void scatter_chunks(const int32_t* pre, const int32_t* __restrict__ cp,
                                      const BatchSched* S, int M, int faces, Key key,
                                      const int32_t* __restrict__ offs, Writer out, int* base,
                                      int b, int nbk) {
  const int lane = threadIdx.x;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int total = pre[M];
  for (int t = loop_rank(total, b, nbk), n_ = loop_blocks(total, nbk); t < total; t += n_) {
    int m = find_mesh(pre, M, t);
    int j = t - pre[m], nch = cp[m + 1] - cp[m];
    int b0 = faces ? S[m].f0 : S[m].c0;
    int end = b0 + (faces ? S[m].nf : S[m].nc);
    __syncthreads();
    if (lane < kMaxLevels) base[lane] = offs[kMaxLevels * cp[m] + lane * nch + j];
    __syncthreads();
    int first = b0 + j * kChunk;
    for (int step = 0; step < kChunk / 64; ++step) {
      int i = first + step * 64 + lane;
      bool valid = i < end;
      int k_mine = valid ? key(i) : -1;
      unsigned long long pending = __ballot(valid);
      while (pending) {
        int leader = __ffsll(pending) - 1;
        int k = __shfl(k_mine, leader, 64);
        unsigned long long msk = __ballot(k_mine == k);
        int p0 = base[k];
        if (k_mine == k) out(p0 + __popcll(msk & lt), i, k);
        __syncthreads();
        if (lane == leader) base[k] = p0 + __popcll(msk);
        __syncthreads();
        pending &= ~msk;
      }
    }
  }
}

template <typename Key, typename FWriter, typename CWriter>
__global__ __launch_bounds__(64) void k_b_part_scatter(const int32_t* __restrict__ rpf,
                                                       const int32_t* __restrict__ rpc,
                                                       const int32_t* __restrict__ fcp,
                                                       const int32_t* __restrict__ ccp,
                                                       const BatchSched* S, int M, Key fkey,
                                                       Key ckey,
                                                       const int32_t* __restrict__ foffs,
                                                       const int32_t* __restrict__ coffs,
                                                       FWriter fout, CWriter cout) {
  const int h = split_half();
  const bool cells = (int)blockIdx.x >= h;  // block-uniform
  STAGE_PREFIX(cells ? rpc : rpf);
  __shared__ int base[kMaxLevels];
  if (cells)
    scatter_chunks(s_pre, ccp, S, M, 0, ckey, coffs, cout, base, (int)blockIdx.x - h,
                   (int)gridDim.x - h);
  else
    scatter_chunks(s_pre, fcp, S, M, 1, fkey, foffs, fout, base, (int)blockIdx.x, h);
}

// ---- per-subiteration schedule ------------------------------------------
// Per mesh (Alg. 2): after a reclassification, dt_min and theta; the
// subiteration's level tau_s (theta at phase 0, else the largest tau <=
// theta with 2^tau dividing the phase); cells with tau <= upd = min(theta,
// ctz(phase + 1)) end their step.  Active counts are prefixes of the
// level-sorted lists.  Then the tile prefixes of the three work classes.
__global__ __launch_bounds__(1024) void k_b_sched(BatchSched* S, int M, int order,
                                                  unsigned long long* flag,
                                                  int32_t* __restrict__ tp) {
  __shared__ int sh[3][1024];
  const int tid = threadIdx.x;
  const bool err_in = *flag != 0ull;
  int carry[3] = {0, 0, 0};
  for (int b = 0; b < M; b += blockDim.x) {
    int m = b + tid;
    int tiles[3] = {0, 0, 0};
    if (m < M) {
      BatchSched& s = S[m];
      bool err = err_in;
      if (s.reclass) {
        double dtm = __longlong_as_double((long long)s.dtbits);
        if (!(dtm > 0.0) || !isfinite(dtm)) {
          err = true;
          atomicOr(flag, 1ull);
        }
        s.dt_min = dtm;
        s.classified = 1;
        int theta = 0;
        for (int u = 0; u < kMaxLevels; ++u) {
          int64_t n = 0;
          for (int g = 0; g < kMaxLevels; ++g) n += s.hist[g * kMaxLevels + u];
          s.cells_per_level[u] = n;
          if (n > 0) theta = u;
        }
        s.theta = theta;
      }
      if (err) {
        s.n_grad = s.n_flux = s.n_gather = 0;
      } else {
        const int ph = s.phase, th = s.theta, s1 = ph + 1;
        const int ts = ph == 0 ? th : min(th, __ffs(ph) - 1);
        const int up = min(th, __ffs(s1) - 1);
        s.tau_s = ts;
        s.upd = up;
        s.n_flux = s.fstart[ts + 1] - s.fstart[0];
        s.n_grad = order == 2 ? s.cstart[ts + 1] - s.cstart[0] : 0;
        s.n_gather = s.cstart[max(ts, up) + 1] - s.cstart[0];
        int64_t u = 0;
        for (int k = 0; k <= up; ++k) u += s.cells_per_level[k];
        s.cell_updates += u;
        s.face_solves += s.n_flux;
        s.subiterations += 1;
        s.phase = s1 & ((1 << th) - 1);
        s.t += s.dt_min;
        tiles[0] = (s.n_grad + kUnit - 1) / kUnit;
        tiles[1] = (s.n_flux + kUnit - 1) / kUnit;
        tiles[2] = (s.n_gather + kUnit - 1) / kUnit;
      }
    }
    for (int w = 0; w < 3; ++w) sh[w][tid] = tiles[w];
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int y[3];
      for (int w = 0; w < 3; ++w) y[w] = tid >= off ? sh[w][tid - off] : 0;
      __syncthreads();
      for (int w = 0; w < 3; ++w) sh[w][tid] += y[w];
      __syncthreads();
    }
    for (int w = 0; w < 3; ++w) {
      if (m < M) tp[w * (M + 1) + m] = carry[w] + sh[w][tid] - tiles[w];
      carry[w] += sh[w][1023];
    }
    __syncthreads();
  }
  if (tid < 3) tp[tid * (M + 1) + M] = carry[tid];
}

// ---- work kernels -----------------------------------------------------------
// The active work of a subiteration is counted in units of one wave (64
// items).  A block of BS threads takes BS / 64 consecutive units at a time;
// each wave finds the mesh of its unit.  Gradient and cell kernels:
// PERSIST = true walks the units with a fixed grid (prefix in LDS); false
// takes one group of units per block over a grid of the static unit count
// (prefix searched in global memory).  The autotuner picks BS, the grid
// and the grab.

template <typename T, bool PERSIST, int BS>
__global__ __launch_bounds__(BS) void k_b_grad(const int32_t* __restrict__ tp,
                                               const BatchSched* S, int M, int grab,
                                               GradArgs<T> a) {
  constexpr int Q = BS / kUnit;
  __shared__ T sStage[Q][kStageVals];
  const int wv = threadIdx.x / kUnit, lane = threadIdx.x % kUnit;
  // a unit's lane 0 always has an item; the other lanes without one repeat it
  if (PERSIST) {
    STAGE_PREFIX(tp);
    const int total = s_pre[M];
    const int groups = (total + Q - 1) / Q;
    TILE_LOOP(groups, grab) {
      const int u = t * Q + wv;
      if (u < total) {
        int m = find_mesh(s_pre, M, u);
        int j0 = (u - s_pre[m]) * kUnit, j = j0 + lane;
        bool valid = j < S[m].n_grad;
        grad_item<T>(a, a.list[S[m].c0 + (valid ? j : j0)], valid, sStage[wv]);
      }
    }
  } else {
    const int total = tp[M], u0 = loop_rank((total + Q - 1) / Q) * Q, u = u0 + wv;
    if (u >= total) return;  // no barrier follows
    int m = mesh_after(tp, find_mesh(tp, M, u0), u);
    int j0 = (u - tp[m]) * kUnit, j = j0 + lane;
    bool valid = j < S[m].n_grad;
    grad_item<T>(a, a.list[S[m].c0 + (valid ? j : j0)], valid, sStage[wv]);
  }
}

// The flux kernels take one group of 4 units per 256-thread block (grid =
// the static count of face units; waves past the active total skip the
// solve): a persistent loop around the face solve raised its register count
// by a quarter and cost a wave of occupancy.
template <int ORDER, typename T, bool G14>
__global__ __launch_bounds__(kBlock) void k_b_flux(const int32_t* __restrict__ tp,
                                                   const BatchSched* S, int M, FluxArgs<T> a) {
  constexpr int Q = kBlock / kUnit;
  const int total = tp[M];
  const int u0 = loop_rank((total + Q - 1) / Q) * Q;
  if (u0 >= total) return;  // the whole block
  const int u = u0 + (int)(threadIdx.x / kUnit);
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  if (u < total) {
    int m = mesh_after(tp, find_mesh(tp, M, u0), u);
    int j = (u - tp[m]) * kUnit + (int)(threadIdx.x % kUnit);
    if (j < S[m].n_flux)
      flux_store_item<ORDER, T, G14>(a, nt_rec(a.rec + S[m].f0 + j), S[m].dt_min, info, i0, i1,
                                     i2);
  }
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

template <int ORDER, typename T, int FEAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kFeatWaves<T>)))
void k_b_flux_feat(const int32_t* __restrict__ tp, const BatchSched* S, int M, FluxArgs<T> a) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[(FEAT & 2) ? (kBlock / 64) * kMlpFwdLds : 8];
  constexpr int Q = kBlock / kUnit;
  const int total = tp[M];
  const int u0 = loop_rank((total + Q - 1) / Q) * Q;
  if (u0 >= total) return;  // the whole block
  const int u = u0 + (int)(threadIdx.x / kUnit);
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  double i0 = 0, i1 = 0, i2 = 0;
  if (u < total) {  // wave-uniform: the network pass sees all 64 lanes
    int m = mesh_after(tp, find_mesh(tp, M, u0), u);
    int j = (u - tp[m]) * kUnit + (int)(threadIdx.x % kUnit);
    const bool valid = j < S[m].n_flux;
    int4 r = valid ? nt_rec(a.rec + S[m].f0 + j) : make_int4(0, 0, -1, 0);
    flux_feat_item<ORDER, T, FEAT>(a, valid, r, S[m].dt_min,
                                   lds + (threadIdx.x >> 6) * kMlpFwdLds, info, i0, i1, i2);
  }
  flush_counters(info, i0, i1, i2, a.dcount, a.dimpulse);
}

template <typename T, bool PERSIST, int BS>
__global__ __launch_bounds__(BS) void k_b_gather(const int32_t* __restrict__ tp,
                                                 const BatchSched* S, int M, int grab, int NC,
                                                 const int* __restrict__ list,
                                                 const uint32_t* __restrict__ fpack,
                                                 const int* __restrict__ c2f,
                                                 const T* __restrict__ Q,
                                                 const double* __restrict__ vol,
                                                 double* __restrict__ U, double* __restrict__ R,
                                                 unsigned long long* flag) {
  constexpr int QU = BS / kUnit;
  const int wv = threadIdx.x / kUnit, lane = threadIdx.x % kUnit;
  if (PERSIST) {
    STAGE_PREFIX(tp);
    const int total = s_pre[M];
    const int groups = (total + QU - 1) / QU;
    TILE_LOOP(groups, grab) {
      const int u = t * QU + wv;
      if (u < total) {
        int m = find_mesh(s_pre, M, u);
        int j = (u - s_pre[m]) * kUnit + lane;
        if (j < S[m].n_gather)
          if (!cell_gather_item<T>(list[S[m].c0 + j], NC, fpack, c2f, Q, S[m].dt_min, vol, U, R,
                                   S[m].tau_s, S[m].upd))
            atomicOr(flag, 1ull);
      }
    }
  } else {
    const int total = tp[M], u0 = loop_rank((total + QU - 1) / QU) * QU, u = u0 + wv;
    if (u >= total) return;  // no barrier follows
    int m = mesh_after(tp, find_mesh(tp, M, u0), u);
    int j = (u - tp[m]) * kUnit + lane;
    if (j < S[m].n_gather)
      if (!cell_gather_item<T>(list[S[m].c0 + j], NC, fpack, c2f, Q, S[m].dt_min, vol, U, R,
                               S[m].tau_s, S[m].upd))
        atomicOr(flag, 1ull);
  }
}

// one mesh's schedule entry back to "state just set"; keep_counters keeps
// the cumulative counters (state reset)
__global__ void k_b_reset_mesh(BatchSched* S, int m0, int count, int keep_counters) {
  const int m = m0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= m0 + count) return;
  BatchSched& s = S[m];
  s.phase = 0;
  s.theta = 0;
  s.classified = 0;
  s.reclass = 0;
  s.dt_min = 0.0;
  s.t = 0.0;
  s.n_grad = s.n_flux = s.n_gather = 0;
  if (!keep_counters) {
    s.subiterations = 0;
    s.cell_updates = 0;
    s.face_solves = 0;
    for (int k = 0; k < kMaxLevels; ++k) s.cells_per_level[k] = 0;
  }
}

__global__ void k_b_set_levels(BatchSched* S, int m, int L) {
  if (threadIdx.x == 0) {
    S[m].L = L;
    S[m].classified = 0;
  }
}

__global__ void k_b_zero_rows(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---- host side ---------------------------------------------------------------

#define B_TRY(c, expr)                                       \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_error((c), e_, #expr); \
  } while (0)

inline int nblk(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

int cu_count(tafv_ctx* c) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, c->device) != hipSuccess) return 256;
  return std::max(1, p.multiProcessorCount);
}

std::string arch_name(tafv_ctx* c) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, c->device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  size_t k = a.find(':');
  return k == std::string::npos ? a : a.substr(0, k);
}

// Merge the uploaded meshes: cells, faces and half-face ids offset by each
// mesh's segment; [k][n] arrays re-laid as [k][N] over the merged counts;
// boundary markers -(f+1) keep pointing at the mesh's own faces.
void merge_hosts(const std::vector<HostMesh*>& hs, HostMesh& out, std::vector<int64_t>& c0,
                 std::vector<int64_t>& f0) {
  int64_t NC = 0, NF = 0;
  c0.clear();
  f0.clear();
  for (const HostMesh* h : hs) {
    c0.push_back(NC);
    f0.push_back(NF);
    NC += h->nc;
    NF += h->nf;
  }
  out.nc = NC;
  out.nf = NF;
  out.nbnd = 0;
  out.ncolours = 0;
  out.fhL.resize(NF);
  out.fhR.resize(NF);
  out.fcol.resize(NF);
  out.fA.resize(3 * NF);
  out.nb.resize(4 * NC);
  out.c2f.resize(4 * NC);
  out.grc.resize(12 * NC);
  out.vol.resize(NC);
  out.perm.resize(NC);
  for (size_t q = 0; q < hs.size(); ++q) {
    const HostMesh& h = *hs[q];
    const int64_t cb = c0[q], fb = f0[q];
    out.nbnd += h.nbnd;
    out.ncolours = std::max(out.ncolours, h.ncolours);
    for (int64_t f = 0; f < h.nf; ++f) {
      out.fhL[fb + f] = h.fhL[f] + (int32_t)(4 * cb);
      out.fhR[fb + f] = h.fhR[f] >= 0 ? h.fhR[f] + (int32_t)(4 * cb) : -1;
      out.fcol[fb + f] = h.fcol[f];
      for (int k = 0; k < 3; ++k) out.fA[k * NF + fb + f] = h.fA[k * h.nf + f];
    }
    for (int64_t i = 0; i < h.nc; ++i) {
      for (int m = 0; m < 4; ++m) {
        int32_t n = h.nb[m * h.nc + i];
        out.nb[m * NC + cb + i] = n >= 0 ? n + (int32_t)cb : n - (int32_t)fb;
        out.c2f[m * NC + cb + i] = h.c2f[m * h.nc + i] + (int32_t)fb;
      }
      for (int k = 0; k < 12; ++k) out.grc[k * NC + cb + i] = h.grc[k * h.nc + i];
      out.vol[cb + i] = h.vol[i];
      out.perm[cb + i] = h.perm[i];  // local: caller order within the mesh
    }
  }
}

// The merged mesh, schedule table, tile prefixes and capture stream of a
// batch; after a failed build they are released, so that a later call can
// build again.
void release_tables(tafv_ctx* c, Batch& B) {
  for (void** p : {(void**)&B.dsched, (void**)&B.ct, (void**)&B.ft, (void**)&B.cc, (void**)&B.fc,
                   (void**)&B.cnt_f, (void**)&B.cnt_c, (void**)&B.tp, (void**)&B.rp,
                   (void**)&B.tmin, (void**)&B.thist}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  if (B.m) free_dev_mesh(c, B.m);
  B.m = nullptr;
  if (B.cap) (void)hipStreamDestroy(B.cap);
  B.cap = nullptr;
}

tafv_status build_merged(tafv_ctx* c) {
  Batch& B = *c->batch;
  if (B.hosts.empty()) return set_error(c, TAFV_E_ORDER, "no mesh uploaded");
  B_TRY(c, hipSetDevice(c->device));
  const int M = (int)B.hosts.size();
  HostMesh merged;
  std::vector<int64_t> c0, f0;
  merge_hosts(B.hosts, merged, c0, f0);
  if (merged.nc > INT32_MAX / 8 || merged.nf > INT32_MAX / 8)
    return set_error(c, TAFV_E_ARG, "batch too large for 32-bit ids");
  if (M > kMaxBatchMeshes) return set_error(c, TAFV_E_ARG, "too many meshes in one batch");
  DevMesh* dm = nullptr;
  tafv_status st = upload_host_mesh(c, merged, &dm);
  if (st != TAFV_OK) return st;
  B.m = dm;
  // schedule table and tile prefixes
  B.hsched.assign(M, BatchSched{});
  std::vector<int32_t> ct(M + 1), ft(M + 1), cc(M + 1), fc(M + 1);
  ct[0] = ft[0] = cc[0] = fc[0] = 0;
  B.lmax = 1;
  for (int m = 0; m < M; ++m) {
    BatchSched& s = B.hsched[m];
    const HostMesh& h = *B.hosts[m];
    s.c0 = (int32_t)c0[m];
    s.nc = (int32_t)h.nc;
    s.f0 = (int32_t)f0[m];
    s.nf = (int32_t)h.nf;
    s.L = B.L[m];
    B.lmax = std::max(B.lmax, (int32_t)B.L[m]);
    ct[m + 1] = ct[m] + nblk(h.nc, kBlock);
    ft[m + 1] = ft[m] + nblk(h.nf, kBlock);
    cc[m + 1] = cc[m] + nblk(h.nc, kChunk);
    fc[m + 1] = fc[m] + nblk(h.nf, kChunk);
  }
  B.n_cc = cc[M];
  B.n_fc = fc[M];
  B.n_ft = ft[M];
  B.n_ct = ct[M];
  B.n_cu = 0;
  B.n_fu = 0;
  for (int m = 0; m < M; ++m) {
    B.n_cu += nblk(B.hsched[m].nc, kUnit);
    B.n_fu += nblk(B.hsched[m].nf, kUnit);
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(dev_alloc(c, &B.dsched, sizeof(BatchSched) * M));
  for (int32_t** p : {&B.ct, &B.ft, &B.cc, &B.fc}) chk(dev_alloc(c, p, sizeof(int32_t) * (M + 1)));
  chk(dev_alloc(c, &B.tp, sizeof(int32_t) * 3 * (M + 1)));
  chk(dev_alloc(c, &B.rp, sizeof(int32_t) * 4 * (M + 1)));
  chk(dev_alloc(c, &B.tmin, sizeof(double) * std::max(B.n_ct, 1)));
  chk(dev_alloc(c, &B.thist, sizeof(int) * kMaxKeys * std::max(B.n_ct, 1)));
  chk(dev_alloc(c, &B.cnt_c, sizeof(int32_t) * kMaxLevels * std::max(B.n_cc, 1)));
  chk(dev_alloc(c, &B.cnt_f, sizeof(int32_t) * kMaxLevels * std::max(B.n_fc, 1)));
  if (e != hipSuccess) return hip_error(c, e, "batch allocation");
  B_TRY(c, hipMemcpy(B.dsched, B.hsched.data(), sizeof(BatchSched) * M, hipMemcpyHostToDevice));
  B_TRY(c, hipMemcpy(B.ct, ct.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice));
  B_TRY(c, hipMemcpy(B.ft, ft.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice));
  B_TRY(c, hipMemcpy(B.cc, cc.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice));
  B_TRY(c, hipMemcpy(B.fc, fc.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice));
  B_TRY(c, launch_fill_u64(c->stream, B.m->dcount, 0ull, kCounterWords));
  B_TRY(c, launch_fill_u64(c->stream, B.m->dnewton, 0ull, kCounterSlots * kNewtonWords));
  B_TRY(c, launch_fill_f64(c->stream, B.m->dimpulse, 0.0, kCounterWords));
  B_TRY(c, launch_fill_u64(c->stream, B.m->dscal, 0ull, 4));
  B_TRY(c, launch_fill_f64(c->stream, B.m->U, 0.0, (int64_t)5 * merged.nc));
  B_TRY(c, launch_fill_f64(c->stream, B.m->R, 0.0, (int64_t)5 * merged.nc));
  B_TRY(c, hipStreamSynchronize(c->stream));
  B_TRY(c, hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
  B.nmesh = M;
  B.has_state.assign(M, 0);
  for (HostMesh* h : B.hosts) delete h;
  B.hosts.clear();
  B.built = true;
  const int cu = cu_count(c);
  for (int w = 0; w < 3; ++w) B.set[w] = LaunchSet{kStaticBlocksPerCU * cu, 1, kBlock};
  B.set[1] = LaunchSet{std::max((B.n_fu + kBlock / kUnit - 1) / (kBlock / kUnit), 1), 1, kBlock};
  return TAFV_OK;
}

tafv_status build(tafv_ctx* c) {
  if (c->batch->built) return TAFV_OK;
  tafv_status st = build_merged(c);
  if (st != TAFV_OK) release_tables(c, *c->batch);
  return st;
}

FluxFeatures features(tafv_ctx* c) {
  FluxFeatures ft;
  bool mlp = c->prm.guess == TAFV_GUESS_MLP;
  ft.feat = (c->prm.guess_stats ? 1 : 0) | (mlp ? 2 : 0);
  ft.mlp = (const MlpDev*)c->mlp_w;
  ft.guess_gate = (float)c->prm.guess_gate;
  ft.guess_strength = (float)c->prm.guess_strength;
  return ft;
}

StepArgs step_args(tafv_ctx* c) {
  StepArgs a;
  a.gas = make_gas(c->prm.gamma);
  a.cfl = c->prm.cfl;
  a.newton_tol = c->prm.newton_tol;
  a.level_margin = c->prm.level_margin;
  a.dt_min = 0.0;
  a.newton_max_iter = c->prm.newton_max_iter;
  a.boundary = c->prm.boundary;
  a.max_levels = c->batch->lmax;
  a.precision = c->prm.precision;
  a.order = c->prm.order;
  return a;
}

// ---- launches of one subiteration ------------------------------------------

struct Ptrs {
  unsigned long long* dcount;
  double* dimpulse;
  double* U;
  double* R;
  const int32_t* tp;  // work tile prefixes [3][M + 1]
  const BatchSched* S;
  unsigned long long* dnewton;  // Newton-update histogram (null: not kept)
};

hipError_t run_reclass(tafv_ctx* c, hipStream_t s) {
  Batch& B = *c->batch;
  DevMesh& m = *B.m;
  const int M = B.nmesh, G = kReclassBlocksPerCU * cu_count(c);
  const size_t lds = sizeof(int32_t) * (M + 1);
  const int32_t *rc = B.rp, *rf = B.rp + (M + 1), *rcc = B.rp + 2 * (M + 1),
                *rfc = B.rp + 3 * (M + 1);
  unsigned long long* flag = m.dscal + 2;
  hipLaunchKernelGGL(k_b_begin, dim3(1), dim3(1024), 0, s, B.dsched, M, c->prm.reclassify, B.ct,
                     B.ft, B.cc, B.fc, B.rp);
  hipLaunchKernelGGL(k_b_dt, dim3(G), dim3(kBlock), lds, s, rc, B.dsched, M, m.nc, m.nf, m.U,
                     m.vol, m.c2f, m.fA, c->prm.gamma, c->prm.cfl, m.dt, B.tmin, flag);
  hipLaunchKernelGGL(k_b_reduce, dim3(M), dim3(kReduceThreads), 0, s, rc, B.dsched, M, B.tmin,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_b_classify, dim3(G), dim3(kBlock), lds, s, rc, B.dsched, M, m.nc, m.dt,
                     c->prm.level_margin, m.nb_, m.lev);
  // the classification took the first of the L - 1 lowering sweeps
  for (int k = 1; k < B.lmax - 1; ++k)
    hipLaunchKernelGGL(k_b_sweep, dim3(G), dim3(kBlock), lds, s, rc, B.dsched, M, m.nc, k,
                       m.nb_, m.lev);
  // the cell and the face classes of the next steps share a launch, each
  // in one half of a grid twice the size (split_half)
  hipLaunchKernelGGL(k_b_keys, dim3(2 * G), dim3(kBlock), lds, s, rc, rf, B.dsched, M, m.nc,
                     m.nb_, m.lev, m.ckey, m.fpack, B.thist, m.fhL, m.fhR, m.fkey);
  hipLaunchKernelGGL(k_b_cell_early, dim3(G), dim3(kBlock), lds, s, rc, B.dsched, M, m.nc, m.nb_,
                     m.lev, m.ckey, m.fpack, c->prm.order);
  hipLaunchKernelGGL(k_b_reduce, dim3(M), dim3(kReduceThreads), 0, s, rc, B.dsched, M, nullptr,
                     B.thist);
  const int PG = 4 * G;  // 64-thread blocks
  hipLaunchKernelGGL(k_b_part_count<ByteKey>, dim3(2 * PG), dim3(64), lds, s, rfc, rcc, B.fc,
                     B.cc, B.dsched, M, ByteKey{m.fkey}, ByteKey{m.ckey}, B.cnt_f, B.cnt_c);
  hipLaunchKernelGGL(k_b_part_scan, dim3(2 * M), dim3(256), 0, s, B.fc, B.cc, B.dsched, M,
                     B.cnt_f, B.cnt_c);
  hipLaunchKernelGGL((k_b_part_scatter<ByteKey, FaceWriter, IndexWriter>), dim3(2 * PG), dim3(64),
                     lds, s, rfc, rcc, B.fc, B.cc, B.dsched, M, ByteKey{m.fkey}, ByteKey{m.ckey},
                     B.cnt_f, B.cnt_c, FaceWriter{m.frec, m.fhL, m.fhR},
                     IndexWriter{m.pc.list});
  hipLaunchKernelGGL(k_b_sched, dim3(1), dim3(1024), 0, s, B.dsched, M, c->prm.order, flag, B.tp);
  return hipGetLastError();
}

// grab 0: one group of units per block over the static count of cell units
dim3 work_grid(const Batch& B, const LaunchSet& ls) {
  const int q = ls.bs / kUnit;
  return dim3(ls.grab == 0 ? std::max((B.n_cu + q - 1) / q, 1) : ls.grid);
}

// launches kernel template K<PERSIST, BS> for the block size and mode of ls
template <typename Launch>
hipError_t by_shape(const LaunchSet& ls, Launch launch) {
  const bool p = ls.grab != 0;
  switch (ls.bs) {
    case 64: p ? launch.template go<true, 64>() : launch.template go<false, 64>(); break;
    case 128: p ? launch.template go<true, 128>() : launch.template go<false, 128>(); break;
    case 512: p ? launch.template go<true, 512>() : launch.template go<false, 512>(); break;
    default: p ? launch.template go<true, 256>() : launch.template go<false, 256>(); break;
  }
  return hipGetLastError();
}

template <typename T>
struct GradLaunch {
  hipStream_t s;
  dim3 g;
  size_t lds;
  const int32_t* tp;
  const BatchSched* S;
  int M, grab;
  GradArgs<T> a;
  template <bool P, int BS>
  void go() const {
    hipLaunchKernelGGL((k_b_grad<T, P, BS>), g, dim3(BS), P ? lds : 0, s, tp, S, M, grab, a);
  }
};

hipError_t run_grad(tafv_ctx* c, hipStream_t s, const LaunchSet& ls, const Ptrs& p) {
  Batch& B = *c->batch;
  DevMesh& m = *B.m;
  if (c->prm.order != 2) return hipSuccess;
  const int M = B.nmesh;
  const double gm1 = c->prm.gamma - 1.0;
  const dim3 g = work_grid(B, ls);
  const size_t lds = sizeof(int32_t) * (M + 1);
  if (c->prm.precision == TAFV_FP32_FLUX) {
    GradArgs<float> a{m.pc.list, 0, m.nc, m.nf, m.U, m.nb_, m.grc32, m.fA, (float*)m.Wf,
                      gm1, c->prm.boundary};
    return by_shape(ls, GradLaunch<float>{s, g, lds, p.tp, p.S, M, ls.grab, a});
  }
  GradArgs<double> a{m.pc.list, 0, m.nc, m.nf, m.U, m.nb_, m.grc, m.fA, (double*)m.Wf,
                     gm1, c->prm.boundary};
  return by_shape(ls, GradLaunch<double>{s, g, lds, p.tp, p.S, M, ls.grab, a});
}

template <typename T>
void flux_dispatch(hipStream_t s, const Batch& B, int order, int feat, bool g14, int grid,
                   const FluxArgs<T>& f) {
  const int32_t* tp = B.tp + (B.nmesh + 1);
  dim3 g(grid), b(kBlock);
  const int M = B.nmesh;
#define B_FEAT(O, F) hipLaunchKernelGGL((k_b_flux_feat<O, T, F>), g, b, 0, s, tp, B.dsched, M, f)
#define B_PLAIN(O, G) hipLaunchKernelGGL((k_b_flux<O, T, G>), g, b, 0, s, tp, B.dsched, M, f)
  if (feat && g14) {
    if (order == 2) {
      if (feat == 1) B_FEAT(2, 1);
      else if (feat == 2) B_FEAT(2, 2);
      else B_FEAT(2, 3);
    } else {
      if (feat == 1) B_FEAT(1, 1);
      else if (feat == 2) B_FEAT(1, 2);
      else B_FEAT(1, 3);
    }
  } else if (g14) {
    if (order == 2) B_PLAIN(2, true);
    else B_PLAIN(1, true);
  } else {
    if (order == 2) B_PLAIN(2, false);
    else B_PLAIN(1, false);
  }
#undef B_FEAT
#undef B_PLAIN
}

hipError_t run_flux(tafv_ctx* c, hipStream_t s, const Ptrs& p) {
  Batch& B = *c->batch;
  const int grid = std::max((B.n_fu + kBlock / kUnit - 1) / (kBlock / kUnit), 1);
  DevMesh& m = *B.m;
  StepArgs a = step_args(c);
  FluxFeatures ft = features(c);
  if (c->prm.precision == TAFV_FP32_FLUX) {
    FluxArgs<float> f{m.frec, 0, m.nf, m.nc, m.fA32, m.U, (const float*)m.Wf, m.R, (float*)m.Q,
                      p.dcount, p.dimpulse, a, ft.mlp, nullptr, nullptr, 0, 0.0, 0, 0,
                      ft.guess_gate, ft.guess_strength};
    f.dnewton = (ft.feat & 1) ? p.dnewton : nullptr;
    flux_dispatch<float>(s, B, c->prm.order, ft.feat, a.gas.is14, grid, f);
  } else {
    FluxArgs<double> f{m.frec, 0, m.nf, m.nc, m.fA, m.U, (const double*)m.Wf, m.R, (double*)m.Q,
                       p.dcount, p.dimpulse, a, ft.mlp, nullptr, nullptr, 0, 0.0, 0, 0,
                       ft.guess_gate, ft.guess_strength};
    f.dnewton = (ft.feat & 1) ? p.dnewton : nullptr;
    flux_dispatch<double>(s, B, c->prm.order, ft.feat, a.gas.is14, grid, f);
  }
  return hipGetLastError();
}

template <typename T>
struct GatherLaunch {
  hipStream_t s;
  dim3 g;
  size_t lds;
  const int32_t* tp;
  const BatchSched* S;
  int M, grab, NC;
  const int *list, *c2f;
  const uint32_t* fpack;
  const T* Q;
  const double* vol;
  double *U, *R;
  unsigned long long* flag;
  template <bool P, int BS>
  void go() const {
    hipLaunchKernelGGL((k_b_gather<T, P, BS>), g, dim3(BS), P ? lds : 0, s, tp, S, M, grab, NC,
                       list, fpack, c2f, Q, vol, U, R, flag);
  }
};

hipError_t run_gather(tafv_ctx* c, hipStream_t s, const LaunchSet& ls, const Ptrs& p) {
  Batch& B = *c->batch;
  DevMesh& m = *B.m;
  const int M = B.nmesh;
  const dim3 g = work_grid(B, ls);
  const size_t lds = sizeof(int32_t) * (M + 1);
  const int32_t* tp = p.tp + 2 * (M + 1);
  unsigned long long* flag = m.dscal + 2;
  if (c->prm.precision == TAFV_FP32_FLUX)
    return by_shape(ls, GatherLaunch<float>{s, g, lds, tp, p.S, M, ls.grab, m.nc, m.pc.list,
                                            m.c2f, m.fpack, (const float*)m.Q, m.vol, p.U, p.R,
                                            flag});
  return by_shape(ls, GatherLaunch<double>{s, g, lds, tp, p.S, M, ls.grab, m.nc, m.pc.list,
                                           m.c2f, m.fpack, (const double*)m.Q, m.vol, p.U, p.R,
                                           flag});
}

Ptrs live_ptrs(Batch& B) {
  return Ptrs{B.m->dcount, B.m->dimpulse, B.m->U, B.m->R, B.tp, B.dsched, B.m->dnewton};
}

// one subiteration on stream s (profiling scopes only when s is the
// context stream and nothing is being captured)
hipError_t run_subiteration(tafv_ctx* c, hipStream_t s, bool prof) {
  Batch& B = *c->batch;
  Ptrs p = live_ptrs(B);
  hipError_t e;
  {
    ProfScope ps(prof ? c : nullptr, P_CLASSIFY, B.m->nc);
    e = run_reclass(c, s);
    if (e != hipSuccess) return e;
  }
  {
    ProfScope ps(prof ? c : nullptr, P_GRAD, 0);
    e = run_grad(c, s, B.set[0], p);
    if (e != hipSuccess) return e;
  }
  {
    ProfScope ps(prof ? c : nullptr, P_FLUX, 0);
    e = run_flux(c, s, p);
    if (e != hipSuccess) return e;
  }
  ProfScope ps(prof ? c : nullptr, P_GATHER, 0);
  return run_gather(c, s, B.set[2], p);
}

// ---- autotuning -------------------------------------------------------------

std::string tune_key(tafv_ctx* c) {
  Batch& B = *c->batch;
  int64_t nc = B.m->nc;
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= nc) ++bucket;
  std::ostringstream o;
  o << arch_name(c) << ":p" << c->prm.precision << ":o" << c->prm.order << ":g" << c->prm.guess
    << ":n" << bucket;
  return o.str();
}

bool cache_lookup(tafv_ctx* c, const std::string& key) {
  Batch& B = *c->batch;
  if (B.cache.empty()) return false;
  std::ifstream f(B.cache);
  if (!f) return false;
  std::string line;
  bool found = false;
  LaunchSet got[3];
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k;
    LaunchSet t[3];
    if (!(in >> k >> t[0].grid >> t[0].grab >> t[0].bs >> t[2].grid >> t[2].grab >> t[2].bs))
      continue;
    if (k != key) continue;
    bool ok = true;
    for (int w : {0, 2})
      ok &= t[w].grid >= 0 && t[w].grab >= 0 && t[w].grab <= 64 &&
            (t[w].bs == 64 || t[w].bs == 128 || t[w].bs == 256 || t[w].bs == 512) &&
            (t[w].grab == 0 || t[w].grid > 0);
    if (!ok) continue;
    for (int w : {0, 2}) got[w] = t[w];
    found = true;  // the last matching line wins
  }
  if (found)
    for (int w : {0, 2}) B.set[w] = got[w];
  return found;
}

void cache_store(tafv_ctx* c, const std::string& key) {
  Batch& B = *c->batch;
  if (B.cache.empty()) return;
  std::ofstream f(B.cache, std::ios::app);
  if (!f) return;
  f << key;
  for (int w : {0, 2}) f << ' ' << B.set[w].grid << ' ' << B.set[w].grab << ' ' << B.set[w].bs;
  f << '\n';
}

tafv_status sync_back(tafv_ctx* c) {
  Batch& B = *c->batch;
  B_TRY(c, hipMemcpyAsync(B.hsched.data(), B.dsched, sizeof(BatchSched) * B.nmesh,
                          hipMemcpyDeviceToHost, c->stream));
  B_TRY(c, hipMemcpyAsync(c->hpin, B.m->dscal, 4 * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, c->stream));
  B_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

// Times candidate launch widths of the gradient and cell kernels on the
// first subiteration's lists (after its flux), over synthetic schedules that
// stand for a whole iteration: for each level tau, every mesh runs its
// subiteration-level-tau work (tau_s = min(tau, theta_m)), weighted by how
// often that level comes up (2^-(tau+1), the top level 2^-theta_max).  The
// gradient kernel rewrites the face values with the same numbers; the cell
// kernel runs on copies of U and R.  Three timed runs after one warm-up per
// candidate and level.
tafv_status autotune(tafv_ctx* c) {
  Batch& B = *c->batch;
  DevMesh& m = *B.m;
  hipStream_t s = c->stream;
  const int M = B.nmesh;
  tafv_status st = sync_back(c);  // lists and levels of this iteration
  if (st != TAFV_OK) return st;
  const int cu = cu_count(c);
  // block sizes 64-512; persistent grids of 8, 16 or 32 waves per CU taking
  // 1 or 4 groups of units at a time, or one group per block
  std::vector<LaunchSet> cand;
  for (int bs : {64, 128, 256, 512}) {
    for (int wpc : {8, 16, 32})
      for (int grab : {1, 4}) cand.push_back(LaunchSet{wpc * cu / (bs / kUnit), grab, bs});
    cand.push_back(LaunchSet{0, 0, bs});
  }
  int theta_max = 0;
  for (const BatchSched& x : B.hsched) theta_max = std::max(theta_max, x.theta);
  const size_t rows = (size_t)5 * m.nc;
  double *Us = nullptr, *Rs = nullptr;
  BatchSched* St = nullptr;
  int32_t* tpt = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = dev_alloc(c, &Us, rows * sizeof(double));
  if (e == hipSuccess) e = dev_alloc(c, &Rs, rows * sizeof(double));
  if (e == hipSuccess) e = dev_alloc(c, &St, sizeof(BatchSched) * M);
  if (e == hipSuccess) e = dev_alloc(c, &tpt, sizeof(int32_t) * 3 * (M + 1));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<double> score[2];
  score[0].assign(cand.size(), 0.0);
  score[1].assign(cand.size(), 0.0);
  std::vector<BatchSched> hs;
  std::vector<int32_t> htp(3 * (M + 1));
  for (int tau = 0; tau <= theta_max && e == hipSuccess; ++tau) {
    const double weight = tau < theta_max ? std::ldexp(1.0, -(tau + 1)) : std::ldexp(1.0, -theta_max);
    hs = B.hsched;
    int acc[3] = {0, 0, 0};
    for (int q = 0; q < M; ++q) {
      BatchSched& x = hs[q];
      const int ts = std::min(tau, x.theta);
      const int up = tau == 0 ? std::min(1, x.theta) : 0;
      x.tau_s = ts;
      x.upd = up;
      x.n_grad = c->prm.order == 2 ? x.cstart[ts + 1] - x.cstart[0] : 0;
      x.n_gather = x.cstart[std::max(ts, up) + 1] - x.cstart[0];
      const int n[3] = {x.n_grad, 0, x.n_gather};
      for (int w = 0; w < 3; ++w) {
        htp[w * (M + 1) + q] = acc[w];
        acc[w] += (n[w] + kUnit - 1) / kUnit;
      }
    }
    for (int w = 0; w < 3; ++w) htp[w * (M + 1) + M] = acc[w];
    e = hipMemcpyAsync(St, hs.data(), sizeof(BatchSched) * M, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tpt, htp.data(), sizeof(int32_t) * 3 * (M + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffers reused next level
    Ptrs scratch{m.dcount, m.dimpulse, Us, Rs, tpt, St, nullptr};
    for (int w = 0; w < 2 && e == hipSuccess; ++w) {
      if (w == 0 && c->prm.order != 2) continue;
      for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k) {
        float tot = 0.f;
        for (int r = 0; r < 4 && e == hipSuccess; ++r) {
          if (w == 1) {
            e = hipMemcpyAsync(Us, m.U, rows * sizeof(double), hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
              e = hipMemcpyAsync(Rs, m.R, rows * sizeof(double), hipMemcpyDeviceToDevice, s);
          }
          if (e == hipSuccess) e = hipEventRecord(e0, s);
          if (e == hipSuccess)
            e = w == 0 ? run_grad(c, s, cand[k], scratch) : run_gather(c, s, cand[k], scratch);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (r > 0) tot += ms;
        }
        score[w][k] += weight * tot;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* ptr : {(void*)Us, (void*)Rs, (void*)St, (void*)tpt}) dev_free(c, ptr);
  if (e != hipSuccess) return hip_error(c, e, "autotuning");
  for (int w = 0; w < 2; ++w) {
    if (w == 0 && c->prm.order != 2) continue;
    size_t best = 0;
    for (size_t k = 1; k < cand.size(); ++k)
      if (score[w][k] < score[w][best]) best = k;
    B.set[w == 0 ? 0 : 2] = cand[best];
  }
  if (c->prm.order != 2) B.set[0] = B.set[2];
  return TAFV_OK;
}

void drop_graphs(Batch& B) {
  for (auto& pe : B.execs) (void)hipGraphExecDestroy(pe.second);
  B.execs.clear();
  B.exec_key = -1;
}

int64_t graph_key(tafv_ctx* c) {
  Batch& B = *c->batch;
  FluxFeatures ft = features(c);
  int64_t k = ft.feat;
  k = k * 16 + B.lmax;
  k = k * 2 + (c->prm.reclassify ? 1 : 0);
  for (int w = 0; w < 3; ++w)
    k = k * 1000003 + (B.set[w].grid * 64 + B.set[w].grab) * 8 + B.set[w].bs / 64;
  return k;
}

tafv_status graph_for(tafv_ctx* c, int64_t len, hipGraphExec_t* out) {
  Batch& B = *c->batch;
  int64_t key = graph_key(c);
  if (key != B.exec_key) {
    drop_graphs(B);
    B.exec_key = key;
  }
  for (auto& pe : B.execs)
    if (pe.first == len) {
      *out = pe.second;
      return TAFV_OK;
    }
  // capture on the context's private stream, replay on the context stream
  B_TRY(c, hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int64_t k = 0; k < len && e == hipSuccess; ++k) e = run_subiteration(c, B.cap, false);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(B.cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_error(c, e != hipSuccess ? e : e2, "graph capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_error(c, e, "graph instantiation");
  B.execs.push_back({len, x});
  *out = x;
  return TAFV_OK;
}


Batch* ready(tafv_ctx* c, int32_t id, tafv_status* st) {
  *st = TAFV_OK;
  Batch& B = *c->batch;
  if (!B.built) {
    *st = build(c);
    if (*st != TAFV_OK) return nullptr;
  }
  if (id < 0 || id >= B.nmesh) {
    *st = set_error(c, TAFV_E_ARG, "unknown mesh");
    return nullptr;
  }
  return &B;
}

}  // namespace

tafv_status batch_upload(tafv_ctx* c, HostMesh* hm, int32_t* mesh_id) {
  Batch& B = *c->batch;
  if (B.built) {
    delete hm;
    return set_error(c, TAFV_E_ORDER, "batched form: meshes must be uploaded before the first state_init");
  }
  *mesh_id = (int32_t)B.hosts.size();
  B.hosts.push_back(hm);
  B.L.push_back(c->prm.max_levels);
  return TAFV_OK;
}

tafv_status batch_mesh_params(tafv_ctx* c, int32_t id, int32_t L) {
  Batch& B = *c->batch;
  if (L < 1 || L > kMaxLevels) return set_error(c, TAFV_E_ARG, "max_levels out of range");
  if (!B.built) {
    if (id < 0 || id >= (int32_t)B.hosts.size()) return set_error(c, TAFV_E_ARG, "unknown mesh");
    B.L[id] = L;
    return TAFV_OK;
  }
  if (id < 0 || id >= B.nmesh) return set_error(c, TAFV_E_ARG, "unknown mesh");
  B_TRY(c, hipSetDevice(c->device));
  B.L[id] = L;
  B.hsched[id].L = L;
  B.hsched[id].classified = 0;
  hipLaunchKernelGGL(k_b_set_levels, dim3(1), dim3(64), 0, c->stream, B.dsched, id, L);
  B_TRY(c, hipGetLastError());
  int32_t lmax = 1;
  for (int32_t v : B.L) lmax = std::max(lmax, v);
  if (lmax != B.lmax) {
    B.lmax = lmax;
    drop_graphs(B);
  }
  return TAFV_OK;
}

tafv_status batch_state_init(tafv_ctx* c, int32_t id, const double* prim) {
  if (!prim) return set_error(c, TAFV_E_ARG, "prim is NULL");
  tafv_status st;
  Batch* Bp = ready(c, id, &st);
  if (!Bp) return st;
  Batch& B = *Bp;
  const BatchSched& s = B.hsched[id];
  for (int64_t i = 0; i < s.nc; ++i) {
    const double* w = prim + 5 * i;
    for (int k = 0; k < 5; ++k)
      if (!std::isfinite(w[k]))
        return set_error(c, TAFV_E_STATE, "non-finite initial value at cell " + std::to_string(i));
    if (!(w[0] > 0.0) || !(w[4] > 0.0))
      return set_error(c, TAFV_E_STATE, "rho <= 0 or p <= 0 at cell " + std::to_string(i));
  }
  B_TRY(c, hipSetDevice(c->device));
  DevMesh& m = *B.m;
  double* xf = m.xfer + 5 * (size_t)s.c0;
  B_TRY(c, hipMemcpyAsync(xf, prim, sizeof(double) * 5 * s.nc, hipMemcpyHostToDevice, c->stream));
  B_TRY(c, launch_state_init_rows(c->stream, s.nc, m.perm + s.c0, xf, c->prm.gamma,
                                  m.U + 5 * (size_t)s.c0, m.R + 5 * (size_t)s.c0));
  B_TRY(c, hipMemcpyAsync(m.U0 + 5 * (size_t)s.c0, m.U + 5 * (size_t)s.c0,
                          sizeof(double) * 5 * s.nc, hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_b_reset_mesh, dim3(1), dim3(64), 0, c->stream, B.dsched, id, 1, 0);
  B_TRY(c, hipGetLastError());
  B_TRY(c, launch_fill_u64(c->stream, m.dscal + 2, 0ull, 1));
  st = sync_back(c);
  if (st != TAFV_OK) return st;
  B.has_state[id] = 1;
  return TAFV_OK;
}

tafv_status batch_state_reset(tafv_ctx* c, int32_t id) {
  tafv_status st;
  if (id == -1) {  // every mesh: one copy of the whole state
    Batch* Bp = ready(c, 0, &st);
    if (!Bp) return st;
    Batch& B = *Bp;
    for (int m = 0; m < B.nmesh; ++m)
      if (!B.has_state[m]) return set_error(c, TAFV_E_ORDER, "no state");
    B_TRY(c, hipSetDevice(c->device));
    DevMesh& dm = *B.m;
    B_TRY(c, hipMemcpyAsync(dm.U, dm.U0, sizeof(double) * 5 * (size_t)dm.nc,
                            hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_b_zero_rows, dim3(nblk((int64_t)5 * dm.nc, 256)), dim3(256), 0,
                       c->stream, dm.R, (int64_t)5 * dm.nc);
    hipLaunchKernelGGL(k_b_reset_mesh, dim3(nblk(B.nmesh, 256)), dim3(256), 0, c->stream,
                       B.dsched, 0, B.nmesh, 1);
    B_TRY(c, hipGetLastError());
    B_TRY(c, launch_fill_u64(c->stream, dm.dscal + 2, 0ull, 1));
    return sync_back(c);
  }
  Batch* Bp = ready(c, id, &st);
  if (!Bp) return st;
  Batch& B = *Bp;
  if (!B.has_state[id]) return set_error(c, TAFV_E_ORDER, "no state");
  B_TRY(c, hipSetDevice(c->device));
  const BatchSched& s = B.hsched[id];
  DevMesh& m = *B.m;
  B_TRY(c, hipMemcpyAsync(m.U + 5 * (size_t)s.c0, m.U0 + 5 * (size_t)s.c0,
                          sizeof(double) * 5 * s.nc, hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_b_zero_rows, dim3(nblk((int64_t)5 * s.nc, 256)), dim3(256), 0, c->stream,
                     m.R + 5 * (size_t)s.c0, (int64_t)5 * s.nc);
  hipLaunchKernelGGL(k_b_reset_mesh, dim3(1), dim3(64), 0, c->stream, B.dsched, id, 1, 1);
  B_TRY(c, hipGetLastError());
  B_TRY(c, launch_fill_u64(c->stream, m.dscal + 2, 0ull, 1));
  return sync_back(c);
}

tafv_status batch_advance(tafv_ctx* c, int64_t n, tafv_stats* out) {
  Batch& B = *c->batch;
  tafv_status st;
  if (!B.built) return set_error(c, TAFV_E_ORDER, "advance before state_init");
  for (int m = 0; m < B.nmesh; ++m)
    if (!B.has_state[m]) return set_error(c, TAFV_E_ORDER, "advance before state_init");
  if (c->prm.guess == TAFV_GUESS_MLP && !c->mlp_ready)
    return set_error(c, TAFV_E_MLP, "learned guess selected but no network set");
  B_TRY(c, hipSetDevice(c->device));
  const std::vector<BatchSched> before = B.hsched;
  int64_t left = n;
  if (left > 0 && B.autotune && B.tuned == 0) {
    if (cache_lookup(c, tune_key(c))) {
      B.tuned = 2;
    } else {
      // first subiteration: reclassify, gradient and flux with the
      // defaults, time the candidates on its lists, then its cell step
      Ptrs p = live_ptrs(B);
      B_TRY(c, run_reclass(c, c->stream));
      B_TRY(c, run_grad(c, c->stream, B.set[0], p));
      B_TRY(c, run_flux(c, c->stream, p));
      st = autotune(c);
      if (st != TAFV_OK) return st;
      B.tuned = 1;
      cache_store(c, tune_key(c));
      B_TRY(c, run_gather(c, c->stream, B.set[2], p));
      --left;
    }
  }
  const bool use_graph = B.graph && !c->profile;
  while (left > 0) {
    int64_t len = std::min<int64_t>(left, kGraphSpan);
    if (use_graph) {
      hipGraphExec_t x = nullptr;
      st = graph_for(c, len, &x);
      if (st != TAFV_OK) return st;
      B_TRY(c, hipGraphLaunch(x, c->stream));
    } else {
      for (int64_t k = 0; k < len; ++k) B_TRY(c, run_subiteration(c, c->stream, c->profile));
    }
    left -= len;
  }
  st = sync_back(c);
  if (st != TAFV_OK) return st;
  const unsigned long long* sc = (const unsigned long long*)c->hpin;
  tafv_stats now{};
  st = read_slot_counters(c, *B.m, &now);
  if (st != TAFV_OK) return st;
  if (out) {
    tafv_stats acc{};
    for (int m = 0; m < B.nmesh; ++m) {
      const BatchSched& a = before[m];
      const BatchSched& b = B.hsched[m];
      acc.subiterations = std::max<int64_t>(acc.subiterations, b.subiterations - a.subiterations);
      acc.cell_updates += b.cell_updates - a.cell_updates;
      acc.face_solves += b.face_solves - a.face_solves;
      acc.theta = std::max(acc.theta, b.theta);
      for (int k = 0; k < kMaxLevels; ++k) acc.cells_per_level[k] += b.cells_per_level[k];
    }
    const BatchSched& last = B.hsched[B.nmesh - 1];
    acc.phase = last.phase;
    acc.dt_min = last.dt_min;
    acc.t_reached = last.t;
    acc.newton_updates = now.newton_updates - B.last.newton_updates;
    acc.newton_fallbacks = now.newton_fallbacks - B.last.newton_fallbacks;
    acc.vacuum_faces = now.vacuum_faces - B.last.vacuum_faces;
    acc.guess_faces = now.guess_faces - B.last.guess_faces;
    acc.guess_newton_updates = now.guess_newton_updates - B.last.guess_newton_updates;
    acc.guess_rejected = now.guess_rejected - B.last.guess_rejected;
    acc.guess_used = now.guess_used - B.last.guess_used;
    acc.guess_evaluated = now.guess_evaluated - B.last.guess_evaluated;
    for (int k = 0; k < 24; ++k)
      acc.newton_hist[k / 8][k % 8] = now.newton_hist[k / 8][k % 8] - B.last.newton_hist[k / 8][k % 8];
    for (int k = 0; k < 3; ++k)
      acc.newton_hist_long_updates[k] =
          now.newton_hist_long_updates[k] - B.last.newton_hist_long_updates[k];
    for (int k = 0; k < 3; ++k) acc.wall_impulse[k] = now.wall_impulse[k] - B.last.wall_impulse[k];
    *out = acc;
  }
  B.last = now;
  if (sc[2]) return set_error(c, TAFV_E_NUMERIC, "non-finite or non-physical cell state");
  return TAFV_OK;
}

tafv_status batch_mesh_stats(tafv_ctx* c, int32_t id, tafv_stats* out) {
  if (!out) return set_error(c, TAFV_E_ARG, "out is NULL");
  tafv_status st;
  Batch* Bp = ready(c, id, &st);
  if (!Bp) return st;
  const BatchSched& s = Bp->hsched[id];
  tafv_stats r{};
  r.subiterations = s.subiterations;
  r.cell_updates = s.cell_updates;
  r.face_solves = s.face_solves;
  for (int k = 0; k < kMaxLevels; ++k) r.cells_per_level[k] = s.cells_per_level[k];
  r.theta = s.theta;
  r.phase = s.phase;
  r.dt_min = s.dt_min;
  r.t_reached = s.t;
  *out = r;
  return TAFV_OK;
}

tafv_status batch_state_read(tafv_ctx* c, int32_t id, double* cons, int8_t* levels) {
  if (!cons) return set_error(c, TAFV_E_ARG, "cons is NULL");
  tafv_status st;
  Batch* Bp = ready(c, id, &st);
  if (!Bp) return st;
  Batch& B = *Bp;
  if (!B.has_state[id]) return set_error(c, TAFV_E_ORDER, "no state");
  B_TRY(c, hipSetDevice(c->device));
  const BatchSched& s = B.hsched[id];
  DevMesh& m = *B.m;
  double* xf = m.xfer + 5 * (size_t)s.c0;
  B_TRY(c, launch_rows_to_caller_f64(c->stream, s.nc, m.perm + s.c0, m.U + 5 * (size_t)s.c0, xf));
  B_TRY(c, hipMemcpyAsync(cons, xf, sizeof(double) * 5 * s.nc, hipMemcpyDeviceToHost, c->stream));
  B_TRY(c, hipStreamSynchronize(c->stream));
  if (levels) {
    int8_t* stage = (int8_t*)xf;
    B_TRY(c, launch_rows_to_caller_i8(c->stream, s.nc, m.perm + s.c0, m.lev + s.c0, stage));
    B_TRY(c, hipMemcpyAsync(levels, stage, s.nc, hipMemcpyDeviceToHost, c->stream));
    B_TRY(c, hipStreamSynchronize(c->stream));
  }
  return TAFV_OK;
}

tafv_status batch_checkpoint_read(tafv_ctx* c, int32_t id, double* cons, double* accum,
                                  int8_t* levels, int32_t* phase, int32_t* theta,
                                  double* dt_min, double* t) {
  if (!accum || !levels || !phase || !theta || !dt_min || !t)
    return set_error(c, TAFV_E_ARG, "NULL argument");
  tafv_status st = batch_state_read(c, id, cons, levels);
  if (st != TAFV_OK) return st;
  Batch& B = *c->batch;
  const BatchSched& s = B.hsched[id];
  DevMesh& m = *B.m;
  double* xf = m.xfer + 5 * (size_t)s.c0;
  B_TRY(c, launch_rows_to_caller_f64(c->stream, s.nc, m.perm + s.c0, m.R + 5 * (size_t)s.c0, xf));
  B_TRY(c, hipMemcpyAsync(accum, xf, sizeof(double) * 5 * s.nc, hipMemcpyDeviceToHost, c->stream));
  B_TRY(c, hipStreamSynchronize(c->stream));
  *phase = s.phase;
  *theta = s.theta;
  *dt_min = s.dt_min;
  *t = s.t;
  return TAFV_OK;
}

tafv_status batch_config(tafv_ctx* c, int32_t graph, int32_t autotune_on, const char* cache) {
  Batch& B = *c->batch;
  if ((graph != 0 && graph != 1) || (autotune_on != 0 && autotune_on != 1))
    return set_error(c, TAFV_E_ARG, "graph and autotune must be 0 or 1");
  B.graph = graph;
  B.autotune = autotune_on;
  B.cache = cache ? cache : "";
  if (!autotune_on && B.built) {
    const int cu = cu_count(c);
    B.set[0] = B.set[2] = LaunchSet{kStaticBlocksPerCU * cu, 1, kBlock};
  }
  B.tuned = 0;
  drop_graphs(B);
  return TAFV_OK;
}

tafv_status batch_info(tafv_ctx* c, int32_t* info, int32_t n) {
  Batch& B = *c->batch;
  if (!info || n < 10) return set_error(c, TAFV_E_ARG, "info needs 10 entries");
  for (int w = 0; w < 3; ++w) {
    info[3 * w] = B.built ? (int32_t)work_grid(B, B.set[w]).x : B.set[w].grid;
    if (w == 1) info[3 * w] = B.set[1].grid;
    info[3 * w + 1] = B.set[w].grab;
    info[3 * w + 2] = B.set[w].bs;
  }
  info[9] = B.tuned;
  return TAFV_OK;
}

void batch_invalidate(tafv_ctx* c) {
  if (c->batch) drop_graphs(*c->batch);
}

void batch_free(tafv_ctx* c) {
  if (!c->batch) return;
  Batch& B = *c->batch;
  drop_graphs(B);
  for (HostMesh* h : B.hosts) delete h;
  release_tables(c, B);
  delete c->batch;
  c->batch = nullptr;
}

}  // namespace tafv
