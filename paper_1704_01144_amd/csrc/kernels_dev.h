// Per-item device functions of the temporal-adaptive finite-volume path
// (Sec. 2.1 Eq. (1) fluxes and sums, Sec. 2.2 Alg. 2 schedule), shared by
// the single-mesh kernels (kernels.hip) and the batched kernels (batch.hip).
// Each function handles one cell or one face; the kernels around them decide
// which items a thread takes.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mlp.h"

namespace tafv {

constexpr int kBlock = 256;
constexpr int kCountSlots = kCounterSlots;
constexpr int kSlotStride = kCounterStride;  // 128 bytes between slots

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD works on runs of kXcdRun consecutive ranks (4096
// items of 256-thread blocks), the runs dealt round-robin to the XCDs: the
// neighbour gathers of a run mostly hit the L2 of its XCD, and work that
// clusters in space (the active cells and faces of a subiteration, the
// faces that need more Newton updates) still spreads over all XCDs.  Runs
// of 1/8 of the launch each (one contiguous range per XCD) left the XCDs
// unevenly loaded; one block per run loses the L2 locality.  Ranks past the
// last whole round of runs keep their index.
constexpr int kXcdRun = 16;
__device__ inline int xcd_rank(int b, int n) {
  const int full = (n / (8 * kXcdRun)) * (8 * kXcdRun);
  if (b >= full) return b;
  const int x = b & 7, i = b >> 3;  // the block's XCD and its index there
  return ((i / kXcdRun) * 8 + x) * kXcdRun + i % kXcdRun;
}
__device__ inline int xcd_block() { return xcd_rank(blockIdx.x, gridDim.x); }

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
// time step, classification, sweeps, keys (phase 0 of an iteration)

// dt_i = cfl V_i / sum_f (|u_i . n_f - xi_f| + a_i) |A_f|, xi_f = sF_f / |A_f|
// the normal speed of a moving face (sF null: a fixed mesh); infinity and
// bad = true on a non-physical state
__device__ inline double dt_item(int i, int nc, int nf, const double* __restrict__ U,
                                 const double* __restrict__ vol, const int* __restrict__ c2f,
                                 const double* __restrict__ fA, double gamma, double cfl,
                                 bool& bad, const double* __restrict__ sF = nullptr) {
  // the face ids, then all 4 area vectors, are requested together
  int f[4];
  for (int m = 0; m < 4; ++m) f[m] = c2f[m * nc + i];
  double w[5];
  cons2prim(U + 5 * (size_t)i, gamma - 1.0, w);
  double A[4][3];
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 3; ++q) A[m][q] = fA[(size_t)q * nf + f[m]];
  double xs[4] = {0, 0, 0, 0};
  if (sF)
    for (int m = 0; m < 4; ++m) xs[m] = sF[f[m]];
  const bool ok = w[0] > 0.0 && w[4] > 0.0 && isfinite(w[4]);
  double a = sqrt(gamma * w[4] / w[0]);
  double s = 0.0;
  for (int m = 0; m < 4; ++m) {
    const double ax = A[m][0], ay = A[m][1], az = A[m][2];
    double am = sqrt(ax * ax + ay * ay + az * az);
    double un = (w[1] * ax + w[2] * ay + w[3] * az) / am;
    if (sF) un -= xs[m] / am;
    s += (fabs(un) + a) * am;
  }
  const double dti = cfl * vol[i] / s;
  if (!ok) {
    bad = true;
    return INFINITY;
  }
  return dti;
}

// tau_i = clamp(floor(log2(dt_i (1 - margin) / dt_min)), 0, L-1) by frexp
__device__ inline int8_t classify_item(double dti, double dtmin, double margin, int L) {
  double q = dti * (1.0 - margin) / dtmin;
  int e;
  frexp(q, &e);
  int t = e - 1;
  t = t < 0 ? 0 : (t > L - 1 ? L - 1 : t);
  return (int8_t)t;
}

// one lowering Jacobi sweep: tau_i <- min(tau_i, min_j tau_j + 1)
// (the neighbour ids, then their levels, are requested together; a boundary
// slot reads the cell's own level and is not used)
__device__ inline int8_t sweep_item(int i, int nc, const int* __restrict__ nb,
                                    const int8_t* __restrict__ src) {
  int n[4], tn[4];
  for (int m = 0; m < 4; ++m) n[m] = nb[m * nc + i];
  for (int m = 0; m < 4; ++m) tn[m] = src[n[m] >= 0 ? n[m] : i];
  int t = src[i];
  for (int m = 0; m < 4; ++m)
    if (n[m] >= 0) t = min(t, tn[m] + 1);
  return (int8_t)t;
}

// per face: tau_f = level of the faster side; key (colour, tau_f) or tau_f
__device__ inline int8_t face_key_item(int f, const int* __restrict__ fhL,
                                       const int* __restrict__ fhR,
                                       const int8_t* __restrict__ fcol,
                                       const int8_t* __restrict__ lev, int use_colour) {
  const int hl = fhL[f], h = fhR[f];
  int t = lev[hl >> 2];
  const int tr = lev[(h >= 0 ? h : hl) >> 2];
  if (h >= 0) t = min(t, tr);
  return (int8_t)(use_colour ? fcol[f] * kMaxLevels + t : t);
}

// per cell: tau_g = lowest level of its faces (the partition key) and the
// packed face word (tau_f per local face in bits 4m, higher-id side bits
// 16 + m, tau in bits 20-23); returns the histogram bin tau_g * 8 + tau
__device__ inline int cell_key_item(int i, int nc, const int* __restrict__ nb,
                                    const int8_t* __restrict__ lev, int8_t* __restrict__ ckey,
                                    uint32_t* __restrict__ fpack) {
  int n4[4], tn[4];
  for (int m = 0; m < 4; ++m) n4[m] = nb[m * nc + i];
  for (int m = 0; m < 4; ++m) tn[m] = lev[n4[m] >= 0 ? n4[m] : i];
  int ti = lev[i], tg = ti;
  uint32_t pk = (uint32_t)ti << 20;
  for (int m = 0; m < 4; ++m) {
    int n = n4[m];
    int tf = n >= 0 ? min(ti, tn[m]) : ti;
    tg = min(tg, tf);
    pk |= (uint32_t)tf << (4 * m);
    if (n >= 0 && n < i) pk |= 1u << (16 + m);
  }
  ckey[i] = (int8_t)tg;
  fpack[i] = pk;
  return tg * kMaxLevels + ti;
}

// Bit of the packed face word marking a cell that applies its fluxes at its
// step's start: all its faces are on its own level (tau_g = tau), so all the
// fluxes of one of its steps are computed at that step's start, and nothing
// reads its state before the step ends -- no face of it is computed mid-step
// and, at second order, no neighbour has a face on a faster level (which
// would compute the neighbour's gradient from this cell's state mid-step).
// Applying them at the start gives the same bits as accumulating them and
// applying the sum at the end.
constexpr uint32_t kEarlyBit = 1u << 24;

__device__ inline bool cell_early_item(int i, int nc, const int* __restrict__ nb,
                                       const int8_t* __restrict__ lev,
                                       const int8_t* __restrict__ ckey,
                                       uint32_t* __restrict__ fpack, int order) {
  if (order == 0) return false;
  const int t = lev[i];
  bool e = ckey[i] == t;
  if (order == 2) {
    int n[4], kn[4];
    for (int m = 0; m < 4; ++m) n[m] = nb[m * nc + i];
    for (int m = 0; m < 4; ++m) kn[m] = ckey[n[m] >= 0 ? n[m] : i];
    for (int m = 0; m < 4; ++m)
      if (n[m] >= 0 && kn[m] < t) e = false;
  }
  if (e) fpack[i] |= kEarlyBit;
  return e;
}

// A launch over the first n1 entries of a cell list and the entries from
// off2 on: item idx is list[idx] for idx < n1, else list[off2 + idx - n1].
__device__ inline int list_cell(const int* __restrict__ list, int n1, int off2, int idx) {
  return idx < n1 ? list[idx] : list[off2 + (idx - n1)];
}

// The gather's cell list (single-mesh form) is sorted by the key 2 k + b:
// k = the level for a cell of kEarlyBit (b = 0), k = tau_g for the others
// (b = 1).  Its cells keep the spatial order of the tau_g list, and a launch
// takes a few ranges of it (ListRanges): item idx lies in the last range r
// with cum[r] <= idx.  The scan is unrolled over the fixed number of slots so
// that the ranges stay in scalar registers.
__device__ inline int range_cell(const int* __restrict__ list, const ListRanges& R, int idx) {
  if (!list) return idx;  // a launch over the whole mesh in its own order
  int base = R.off[0];
#pragma unroll
  for (int r = 1; r < kMaxLevels + 1; ++r)
    if (r < R.n && idx >= R.cum[r]) base = R.off[r] - R.cum[r];
  return list[base + idx];
}

// h[bin] += 1 for every active lane, one LDS atomic per distinct bin of the
// wave (lanes with equal bins are counted by a ballot): the bins of a
// histogram by level are few, and per-lane atomics on them serialise
__device__ inline void wave_hist_add(int* h, bool active, int bin) {
  unsigned long long pending = __ballot(active);
  while (pending) {
    const int leader = __ffsll(pending) - 1;
    const int b = __shfl(bin, leader, 64);
    const unsigned long long same = __ballot(active && bin == b);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(&h[b], __popcll(same));
    pending &= ~same;
  }
}

// partition keys and list writers
struct ByteKey {
  const int8_t* key;
  __device__ int operator()(int i) const { return key[i]; }
};

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

// ---------------------------------------------------------------------------
// least-squares gradient + Barth-Jespersen limiter + face reconstruction

template <typename T>
struct GradArgs {
  const int* list;
  int count, nc, nf;
  const double* U;
  const int* nb;
  const T* grc;  // [12][nc] a_mj = c_j . r_m at (4 m + j) nc + cell, m < 3
  const double* fA;
  T* Wf;  // [4][nc][5]: Wf[(slot * nc + cell) * 5 + variable]
  double gm1;
  int boundary;
  const double* sF;  // moving mesh: face volume rates (walls move with them)
  int n1, off2;      // the items are list[0, n1) then list[off2, ...) (see list_cell)
  // list null: the items are the cells i < count with key[i] <= key_max,
  // visited in mesh order
  const int8_t* key;
  int key_max;
  // when set: the face values of the half-faces whose neighbour lies in
  // another chunk of kChunkCells cells go to Wx[xb[cell] + rank of the slot
  // among those of the cell] instead of Wf
  T* Wx = nullptr;
  const int* xb = nullptr;
  // whole-mesh launches: the items are the cells first + idx < count
  int first = 0;
};

// cells per chunk of the compact cross-chunk face values (a block's cells
// in the fused gradient and local-face launch)
constexpr int kChunkCells = 256;

// slots of cell i whose neighbour lies in another chunk
__device__ inline unsigned cross_slots(const int* nb, int i) {
  unsigned x = 0;
  for (int m = 0; m < 4; ++m)
    x |= (unsigned)(nb[m] >= 0 && nb[m] / kChunkCells != i / kChunkCells) << m;
  return x;
}

// Face values are stored per slot and cell with the 5 values of a half-face
// contiguous: Wf[(slot * nc + cell) * 5 + variable], so that the flux kernel
// reads one short run per side.  A wave stages its 4 x 5 x 64 values in LDS
// and then writes each slot with 5 store instructions that cover 64
// consecutive values of the wave's (mostly consecutive) cells, instead of
// 20 instructions whose 64 values lie 40 bytes apart.  All 64 lanes of the
// wave take part; lanes without a cell (valid = false) compute a copy of
// another lane's cell and store nothing.
constexpr int kStageVals = 4 * 5 * 64;  // staging values per wave

template <typename T>
struct FaceValueWriter {
  T* st;  // this wave's staging area, [slot][lane][variable]
  int mine;
  unsigned slots;  // the slots of this lane's cell that are stored (bit m: slot m)
  __device__ FaceValueWriter(T* stage, int i, bool valid, unsigned store_slots = 0xfu)
      : st(stage), mine(valid ? i : -1), slots(store_slots) {}
  __device__ void put(int m, int k, T v) { st[m * 320 + 5 * (threadIdx.x & 63) + k] = v; }
  __device__ void flush(T* __restrict__ Wf, int nc) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = 0; j < 5; ++j) {
      const int d = 64 * j + lane, src = d / 5, kk = d - 5 * src;
      const int cell = __shfl(mine, src, 64);
      const unsigned sl = (unsigned)__shfl((int)slots, src, 64);
      if (cell < 0) continue;
      // non-temporal: the face values are read once, by the next kernel;
      // kept out of the way of the neighbour states in L2
      for (int m = 0; m < 4; ++m)
        if ((sl >> m) & 1u)
          __builtin_nontemporal_store(st[m * 320 + d], &Wf[((size_t)m * nc + cell) * 5 + kk]);
    }
  }
};

// Element at byte offset byte_off of a column that starts at col, the same
// address for the whole wave: the base goes through scalar registers (the
// wave reads it from its first lane) and the load takes one 32-bit offset
// register that all columns of an item share.  Needs byte_off < 2^32, which
// the cell and face counts (< 2^29) guarantee for 8-byte elements.
template <typename T>
__device__ inline T col_load(const T* __restrict__ col, uint32_t byte_off) {
  const uint64_t b = reinterpret_cast<uint64_t>(col);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) T gT;
  gchar* base = (gchar*)(((uint64_t)hi << 32) | lo);
  return *(gT*)(base + byte_off);
}

// Least squares over the 4 face neighbours (mirror ghosts on the boundary):
// G = sum_j c_j (W_j - W_i), used only through its change to the face
// centroids, delta_m = G . r_m = sum_j a_mj (W_j - W_i) with a_mj = c_j . r_m
// (delta_3 = -(delta_0 + delta_1 + delta_2): the offsets r_m of a
// tetrahedron sum to zero).  Barth-Jespersen per variable k: the largest
// psi_k <= 1 keeping W_i + psi_k delta_m inside [min, max] of the cell and
// its neighbours at all 4 face centroids; output W_i + psi_k delta_m.
// All 64 lanes of a wave call this together (see FaceValueWriter); stage:
// kStageVals values.
//
// The loads are grouped so that a cell waits on three dependent trips to
// memory (its list entry; its neighbour ids with its own state and the
// coefficients; the 4 neighbour states together) rather than on two per
// neighbour: a boundary slot loads the cell's own state, which the mirror
// ghost then replaces, so no branch separates the neighbour loads.  The
// sums accumulate neighbour by neighbour, j = 0..3.
// What a cell reads by its own index: neighbour ids, state, coefficients.
template <typename T>
struct GradIn {
  int nb[4];
  double ui[5];
  T cr[3][4];
  int xb;  // the cell's first compact position (GradArgs::Wx set)
};

template <typename T>
__device__ inline GradIn<T> grad_load(const GradArgs<T>& a, int i) {
  const int nc = a.nc;
  const uint32_t o4 = (uint32_t)i * 4u;
  GradIn<T> g;
  for (int j = 0; j < 4; ++j) g.nb[j] = col_load(a.nb + (size_t)j * nc, o4);
  for (int k = 0; k < 5; ++k) g.ui[k] = a.U[5 * (size_t)i + k];
  // the coefficients are read once per item: non-temporal
  for (int m = 0; m < 3; ++m)
    for (int j = 0; j < 4; ++j)
      g.cr[m][j] = __builtin_nontemporal_load(a.grc + (size_t)(4 * m + j) * nc + i);
  g.xb = a.xb ? a.xb[i] : 0;
  return g;
}

// store_slots: the slots whose face values are stored (the others stay in
// the stage only); with a.Wx, the slots across chunks go to the compact
// array instead
template <typename T>
__device__ inline void grad_compute(const GradArgs<T>& a, int i, bool valid, T* stage,
                                    const GradIn<T>& g, unsigned store_slots = 0xfu) {
  const int nc = a.nc;
  const unsigned cross = a.Wx ? cross_slots(g.nb, i) : 0u;
  FaceValueWriter<T> out(stage, i, valid, store_slots & ~cross);
  const int* nb = g.nb;
  const double* ui = g.ui;
  double un[4][5];
  for (int j = 0; j < 4; ++j) {
    const size_t src = 5 * (size_t)(nb[j] >= 0 ? nb[j] : i);
    for (int k = 0; k < 5; ++k) un[j][k] = a.U[src + k];
  }
  const auto& cr = g.cr;
  double wd[5];
  cons2prim(ui, a.gm1, wd);
  T wi[5];
  for (int k = 0; k < 5; ++k) wi[k] = (T)wd[k];
  T dl[3][5], hi[5], lo[5];
  for (int k = 0; k < 5; ++k) dl[0][k] = dl[1][k] = dl[2][k] = hi[k] = lo[k] = 0;
  for (int j = 0; j < 4; ++j) {
    T dw[5];
    double t[5];
    cons2prim(un[j], a.gm1, t);
    for (int k = 0; k < 5; ++k) dw[k] = nb[j] >= 0 ? (T)t[k] - wi[k] : (T)0;
    if (nb[j] < 0 && a.boundary == TAFV_BC_WALL) {
      int f = -nb[j] - 1;
      T ax = (T)a.fA[f], ay = (T)a.fA[a.nf + f], az = (T)a.fA[2 * (size_t)a.nf + f];
      T ia = frsq(ax * ax + ay * ay + az * az);
      T nx = ax * ia, ny = ay * ia, nz = az * ia;
      T vn = wi[1] * nx + wi[2] * ny + wi[3] * nz;
      if (a.sF) vn -= (T)a.sF[f] * ia;  // the wall moves with the face
      T vn2 = 2 * vn;
      dw[1] = -vn2 * nx;
      dw[2] = -vn2 * ny;
      dw[3] = -vn2 * nz;
    }
    for (int k = 0; k < 5; ++k) {
      const T d = dw[k];
      dl[0][k] += cr[0][j] * d;
      dl[1][k] += cr[1][j] * d;
      dl[2][k] += cr[2][j] * d;
      hi[k] = d > hi[k] ? d : hi[k];
      lo[k] = d < lo[k] ? d : lo[k];
    }
  }
  for (int k = 0; k < 5; ++k) {
    const T delta[4] = {dl[0][k], dl[1][k], dl[2][k], -(dl[0][k] + dl[1][k] + dl[2][k])};
    T psi = 1;
    for (int m = 0; m < 4; ++m) {
      const T d = delta[m];
      T phi = 1;
      if (d > 0) phi = hi[k] < d ? hi[k] * frcp(d) : (T)1;
      else if (d < 0) phi = lo[k] > d ? lo[k] * frcp(d) : (T)1;
      psi = phi < psi ? phi : psi;
    }
    for (int m = 0; m < 4; ++m) out.put(m, k, wi[k] + psi * delta[m]);
  }
  out.flush(a.Wf, nc);
  if (valid && cross) {  // this lane's own staged values
    const T* st = stage + 5 * (threadIdx.x & 63);
    T* x = a.Wx + 5 * (size_t)g.xb;
    for (int m = 0; m < 4; ++m) {
      if (!((cross >> m) & 1u)) continue;
      for (int k = 0; k < 5; ++k) x[k] = st[m * 320 + k];
      x += 5;
    }
  }
}

template <typename T>
__device__ inline void grad_item(const GradArgs<T>& a, int i, bool valid, T* stage) {
  grad_compute<T>(a, i, valid, stage, grad_load<T>(a, i));
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
  T* Q;             // gather mode: per-face flux |A| F . n [nf][5]
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
  float guess_strength;  // network only where the jump strength reaches this
  // gather mode, predictor/corrector form: 0 = one pass per face step (store
  // phi; wall impulse dt_f phi); 1 = predictor pass (store phi, no impulse);
  // 2 = corrector pass: store phi0 + phi1 with phi0 from Qpred, the
  // predictor fluxes; wall impulse q = dt_f (phi0 + phi1) / 2
  int pass_mode;
  const T* Qpred;
  const double* sF;  // moving mesh: face volume rates w_f . A_f
  // when set, dt_min is read here on the device (its bit pattern) instead of
  // from s.dt_min: a launch enqueued before the host knows dt_min
  const unsigned long long* dtmin_dev = nullptr;
  // the launch's items: rec[idx] for idx < n1, then rec[off2 + idx - n1]
  // (two ranges of the face list)
  int n1 = 0x7fffffff, off2 = 0;
  // when set: the items of the first range are faces between chunks, their
  // records hold positions in this compact array of face values
  const T* Wx = nullptr;
  // face statistics (FEAT & 1): Newton updates per face by category, in
  // kCountSlots slots of kNewtonWords words (see newton_hist_add)
  unsigned long long* dnewton = nullptr;
  // when set: the launch walks every face in face order (count = nf), and
  // the faces of partition key <= key_max are its items, their records
  // formed from fhL, fhR and the key (tau_f) instead of read from rec
  const int8_t* fkey = nullptr;
  int key_max = 0;
  const int* fhL = nullptr;
  const int* fhR = nullptr;
  int ffirst = 0;  // face-order launches: the faces ffirst + idx < count
};


// whether item idx reads its face values from the compact array
template <typename T>
__device__ inline bool flux_compact(const FluxArgs<T>& a, int idx) {
  return a.Wx != nullptr && idx < a.n1;
}

template <typename T>
__device__ inline const int4* flux_rec(const FluxArgs<T>& a, int idx) {
  return a.rec + (idx < a.n1 ? idx : a.off2 + (idx - a.n1));
}

template <typename T>
__device__ inline double flux_dt_min(const FluxArgs<T>& a) {
  return a.dtmin_dev ? __longlong_as_double((long long)*a.dtmin_dev) : a.s.dt_min;
}

// gather mode: the face's stored flux and the wall impulse of its
// time-integrated flux (phi is replaced by phi0 + phi1 in a corrector pass)
template <typename T>
__device__ inline void store_face_flux(const FluxArgs<T>& a, int4 r, double dt_min, T* phi,
                                       bool wall, double& i0, double& i1, double& i2) {
  double s = 0.0;
  if (a.pass_mode == 2) {
    const T* p0 = a.Qpred + 5 * (size_t)r.x;
    for (int k = 0; k < 5; ++k) phi[k] = (T)((double)p0[k] + (double)phi[k]);
    s = ldexp(dt_min, r.w - 1);
  } else if (a.pass_mode == 0) {
    s = ldexp(dt_min, r.w);
  }
  T* q = a.Q + 5 * (size_t)r.x;
  for (int k = 0; k < 5; ++k) q[k] = phi[k];
  if (wall && a.pass_mode != 1) {
    i0 += s * (double)phi[1];
    i1 += s * (double)phi[2];
    i2 += s * (double)phi[3];
  }
}

template <int ORDER, typename T>
__device__ inline void load_side(const FluxArgs<T>& a, int h, T* w, bool compact = false) {
  if (ORDER == 2) {  // Wf[(slot * nc + cell) * 5 + variable], or Wx[h * 5 + variable]
    const T* p = compact ? a.Wx + 5 * (size_t)h : a.Wf + 5 * ((size_t)(h & 3) * a.nc + (h >> 2));
    for (int k = 0; k < 5; ++k) w[k] = p[k];
  } else {
    double t[5];
    cons2prim(a.U + 5 * (size_t)(h >> 2), a.s.gas.gm1, t);
    for (int k = 0; k < 5; ++k) w[k] = (T)t[k];
  }
}

// Non-temporal loads of what a kernel reads once (face records, face
// areas): they do not displace the states and face values other items of
// the launch read again.  (Face values themselves are read once too, but
// loading them non-temporally made the flux kernel slower.)
template <typename T>
__device__ inline T nt_load(const T* p) {
  return __builtin_nontemporal_load(p);
}
typedef int tafv_i4v __attribute__((ext_vector_type(4)));
__device__ inline int4 nt_rec(const int4* p) {
  const tafv_i4v v = __builtin_nontemporal_load(reinterpret_cast<const tafv_i4v*>(p));
  return make_int4(v.x, v.y, v.z, v.w);
}

// Item idx of a flux launch: its record and whether it is a face to compute.
// A face-order launch requests the key and both half-face ids together.
template <typename T>
__device__ inline bool flux_item(const FluxArgs<T>& a, int idx, int4& r) {
  if (a.fkey) {
    const int fi = a.ffirst + idx;
    const int f = fi < a.count ? fi : a.count - 1;
    const int k = a.fkey[f], hl = a.fhL[f], hr = a.fhR[f];
    r = make_int4(f, hl, hr, k);
    return fi < a.count && k <= a.key_max;
  }
  if (idx >= a.count) {
    r = make_int4(0, 0, -1, 0);
    return false;
  }
  r = nt_rec(flux_rec(a, idx));
  return true;
}

struct SolveInfo {
  int iters, fallback, vacuum;
  int gated, gated_iters, rejected, used;  // faces where two-rarefaction is inexact
  int evaluated;                           // faces the network was evaluated for
};

__device__ inline void add_info(SolveInfo& a, const SolveInfo& b) {
  a.iters += b.iters;
  a.fallback += b.fallback;
  a.vacuum += b.vacuum;
  a.gated += b.gated;
  a.gated_iters += b.gated_iters;
  a.rejected += b.rejected;
  a.used += b.used;
  a.evaluated += b.evaluated;
}

// |A| F(W(0)) . n for one face: reconstructed states, rotation to the face
// normal, exact Riemann solve (p* in FP64), sampling at x/t = 0, flux.
// MOVE: the face moves with normal speed xi = sF / |A| (ALE form): the
// Riemann problem is solved in the face's frame (normal velocities minus
// xi; a wall's mirror state follows the face), sampled at its origin, and
// the flux through the moving face is |A| (F(W) . n - xi U(W)): the
// convective terms take the relative normal velocity, the pressure work the
// absolute one (+ |A| p xi in the energy flux).
// The flux of face f from its two reconstructed states (interior = false: a
// boundary face, wr unused).
template <typename T, bool G14, bool MOVE = false>
__device__ inline void face_flux_w(const FluxArgs<T>& a, int f, bool interior, const T* wl,
                                   const T* wr, T* phi, SolveInfo& info) {
  const Gas& G = a.s.gas;
  T ax = nt_load(a.fA + f), ay = nt_load(a.fA + a.nf + f);
  T az = nt_load(a.fA + 2 * (size_t)a.nf + f);
  T a2 = ax * ax + ay * ay + az * az;
  T ia = frsq(a2);
  T am = a2 * ia;
  T nx = ax * ia, ny = ay * ia, nz = az * ia;
  T unl = wl[1] * nx + wl[2] * ny + wl[3] * nz;
  T xi = 0;
  if (MOVE) {
    xi = (T)a.sF[f] * ia;
    unl -= xi;
  }
  if (!interior && a.s.boundary != TAFV_BC_WALL) {  // transmissive: F(W_L)
    T E = wl[4] * (T)(1.0 / G.gm1) + (T)0.5 * wl[0] * (wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
    phi[0] = am * wl[0] * unl;
    phi[1] = am * (wl[0] * unl * wl[1] + wl[4] * nx);
    phi[2] = am * (wl[0] * unl * wl[2] + wl[4] * ny);
    phi[3] = am * (wl[0] * unl * wl[3] + wl[4] * nz);
    phi[4] = am * unl * (E + wl[4]);
    if (MOVE) phi[4] += am * wl[4] * xi;
    return;
  }
  const bool wall = !interior;
  T unr = wall ? -unl : wr[1] * nx + wr[2] * ny + wr[3] * nz;
  if (MOVE && !wall) unr -= xi;
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
    phi[4] = MOVE ? ps * am * xi : (T)0;  // a moving wall works on the gas
    return;
  }
  T rs, us, ps;
  int side;
  if (G14 && !st.vacuum)
    side = sample14<T>(G, wl[0], unl, wl[4], (T)al, (T)ipl, (T)ral, wr[0], unr, wr[4], (T)ar,
                       (T)ipr, (T)rar, (T)st.p, (T)st.u, rs, us, ps, st.zl, st.zr);
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
  if (MOVE) phi[4] += am * ps * xi;
}

// |A| F(W(0)) . n for one face record (reconstructed states from the face
// values, or the cells' states at first order)
template <int ORDER, typename T, bool G14, bool MOVE = false>
__device__ inline void face_flux(const FluxArgs<T>& a, int4 r, T* phi, SolveInfo& info,
                                 bool compact = false) {
  T wl[5], wr[5];
  load_side<ORDER, T>(a, r.y, wl, compact);
  if (r.z >= 0) load_side<ORDER, T>(a, r.z, wr, compact);
  face_flux_w<T, G14, MOVE>(a, r.x, r.z >= 0, wl, wr, phi, info);
}

// Counters are spread over kCountSlots slots 128 bytes apart (slot = wave
// index modulo kCountSlots) so that the waves of a launch do not all
// serialise on one address; the host sums the slots.  Called by all lanes
// of a wave; each wave adds its sums with its first lane, so the waves of a
// block do not wait for each other.
__device__ inline void flush_counters(const SolveInfo& info, double i0, double i1, double i2,
                                      unsigned long long* dcount, double* dimpulse) {
  int c[8] = {wave_sum(info.iters), wave_sum(info.fallback), wave_sum(info.vacuum),
              wave_sum(info.gated), wave_sum(info.gated_iters), wave_sum(info.rejected),
              wave_sum(info.used), wave_sum(info.evaluated)};
  i0 = wave_sum(i0);
  i1 = wave_sum(i1);
  i2 = wave_sum(i2);
  if ((threadIdx.x & 63) == 0) {
    const int slot = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCountSlots);
    unsigned long long* cs = dcount + slot * kSlotStride;
    for (int k = 0; k < 8; ++k)
      if (c[k]) atomicAdd(&cs[k], (unsigned long long)c[k]);
    if (i0 != 0.0 || i1 != 0.0 || i2 != 0.0) {
      double* d = dimpulse + slot * kSlotStride;
      atomicAdd(&d[0], i0);
      atomicAdd(&d[1], i1);
      atomicAdd(&d[2], i2);
    }
  }
}

// Gather mode: the flux Phi of one face into Q[f], in the flux precision
// (the cells form q = 2^tau_f dt_min Phi in FP64, the same product the
// colour scatter forms); the wall impulse q is added to (i0, i1, i2).
template <int ORDER, typename T, bool G14, bool MOVE = false>
__device__ inline void flux_store_item(const FluxArgs<T>& a, int4 r, double dt_min,
                                       SolveInfo& acc, double& i0, double& i1, double& i2,
                                       bool compact = false) {
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  T phi[5];
  face_flux<ORDER, T, G14, MOVE>(a, r, phi, info, compact);
  add_info(acc, info);
  store_face_flux(a, r, dt_min, phi, r.z < 0 && a.s.boundary == TAFV_BC_WALL, i0, i1, i2);
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
//   FEAT & 2: on those faces whose jump strength |u_R - u_L|/a_m +
//             |p_L - p_R|/p_m reaches guess_strength, the network predicts
//             y ~ ln(p*/p_TR); where |y| exceeds the gate the Newton solve
//             starts from p_TR exp(y) (a non-finite or non-positive guess
//             falls back to p_TR).  The network runs once per wave, on the
//             matrix cores, when any face of the wave passes the strength
//             pre-gate (a few FP32 operations on the two states); only the
//             states are kept across the network pass, the network's inputs
//             are formed for that pass alone, and the two-rarefaction value
//             is formed after it.
// The Newton iteration and its stop test are unchanged, so p* is the same
// root whichever start is used.  All 64 lanes of a wave must call this
// together (valid = false for lanes without a face); wave_lds is this
// wave's kMlpFwdLds elements of LDS.
// Waves per SIMD asked of the kernels that call flux_feat_item: left to
// itself the compiler parks live values in accumulator registers around the
// network pass and settles at 4; the FP32 forms fit 5 without spilling.
template <typename T>
constexpr int kFeatWaves = sizeof(T) == 4 ? 5 : 4;

// The network's inputs for one interior face: the two states' deviations
// from their means, normalised by them (density, normal velocity over the
// mean sound speed, pressure).
template <typename T>
__device__ inline void face_features(const Gas& G, const T* wl, const T* wr, T unl, T unr,
                                     float* x) {
  double rl = wl[0], rr = wr[0], pl = wl[4], pr = wr[4];
  double rm = 0.5 * (rl + rr), pm = 0.5 * (pl + pr);
  double amean = sqrt(G.g * pm / rm);
  double dr = (rl - rr) / (rl + rr), dp = (pl - pr) / (pl + pr);
  double du = 0.5 * ((double)unl - (double)unr) / amean;
  x[0] = (float)dr;
  x[1] = (float)du;
  x[2] = (float)dp;
  x[3] = (float)-dr;
  x[4] = (float)-du;
  x[5] = (float)-dp;
}

// The strength pre-gate |u_R - u_L| / a_m + |p_L - p_R| / p_m >= s of an
// interior face, in FP32 and without a square root or a division: with
// D = s p_m - |p_L - p_R| (p_m times the pressure term's shortfall), it
// holds where D <= 0 or (u_R - u_L)^2 p_m rho_m >= D^2 g
// (a_m^2 = g p_m / rho_m; p_m, rho_m > 0).
template <typename T>
__device__ inline bool strength_pregate(const Gas& G, const T* wl, const T* wr, T unl, T unr,
                                        float s) {
  const float rm = 0.5f * ((float)wl[0] + (float)wr[0]);
  const float pm = 0.5f * ((float)wl[4] + (float)wr[4]);
  const float D = s * pm - fabsf((float)wl[4] - (float)wr[4]);
  if (D <= 0.f) return true;
  const float du = (float)unr - (float)unl;
  return du * du * pm * rm >= D * D * (float)G.g;
}

// Newton updates per face solve by category, per counter slot: word
// 8 c + b counts the solves of category c with b + 1 updates (b < 7) or
// with 8 or more (b = 7), word 24 + c sums the updates of that last bin.
// Category: 0 p* <= min(p_L, p_R) (two rarefactions, the two-rarefaction
// value exact), 1 between them (one shock), 2 above both (two shocks); a
// wall's mirror state has p_R = p_L.  Vacuum faces and transmissive faces
// have no Newton solve and are not counted.  Called by all 64 lanes of a
// wave; key < 0 for lanes without a solve.
__device__ inline void newton_hist_add(unsigned long long* dn, int key, int iters) {
  const int lane = threadIdx.x & 63;
  unsigned long long* d =
      dn + ((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCountSlots) * kNewtonWords;
  unsigned long long pending = __ballot(key >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int k = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(key == k);
    if (lane == leader) atomicAdd(&d[k], (unsigned long long)__popcll(same));
    pending &= ~same;
  }
  if (key >= 0 && (key & 7) == 7) atomicAdd(&d[24 + (key >> 3)], (unsigned long long)iters);
}

// The gather-mode flux with the optional features, as described above, from
// the face's two reconstructed states wl and wr (wr unused on a boundary
// face, r.z < 0); r.x the face, r.w its tau_f.  All 64 lanes of a wave call
// it together; invalid lanes pass any finite states.
template <typename T, int FEAT>
__device__ inline void flux_feat_w(const FluxArgs<T>& a, bool valid, int4 r, const T* wl,
                                   const T* wr, double dt_min, uint16_t* wave_lds,
                                   SolveInfo& acc, double& i0, double& i1, double& i2) {
  const Gas& G = a.s.gas;
  SolveInfo info{0, 0, 0, 0, 0, 0, 0, 0};
  // 1. the face's normal and the strength pre-gate: with the states, all
  // that is kept across the wave's network pass
  T am = 1, nx = 1, ny = 0, nz = 0, unl = 0, unr = 0;
  bool wall = false, transmit = false, net = false;
  float x[kMlpIn] = {0, 0, 0, 0, 0, 0};
  int hist_key = -1, hist_iters = 0;  // face statistics: category and bin
  if (valid) {
    const int f = r.x;
    T ax = nt_load(a.fA + f), ay = nt_load(a.fA + a.nf + f);
    T az = nt_load(a.fA + 2 * (size_t)a.nf + f);
    wall = r.z < 0 && a.s.boundary == TAFV_BC_WALL;
    transmit = r.z < 0 && !wall;
    T a2 = ax * ax + ay * ay + az * az;
    T ia = frsq(a2);
    am = a2 * ia;
    nx = ax * ia;
    ny = ay * ia;
    nz = az * ia;
    unl = wl[1] * nx + wl[2] * ny + wl[3] * nz;
    unr = wall ? -unl : wr[1] * nx + wr[2] * ny + wr[3] * nz;
    if ((FEAT & 2) && r.z >= 0) net = strength_pregate<T>(G, wl, wr, unl, unr, a.guess_strength);
  }
  // 2. the network, once per wave, where any face passes the pre-gate (the
  // inputs are formed only then)
  float ym = 0.f;
  if ((FEAT & 2) && __ballot(net) != 0ull) {
    if (valid && r.z >= 0) face_features<T>(G, wl, wr, unl, unr, x);
    ym = mlp_wave_forward(*a.mlp, x, wave_lds);
  }
  // 3. the face solve: two-rarefaction value, the network's start where the
  // two-rarefaction value is inexact, Newton, sampling, flux
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
      const double rl = wl[0], pl = wl[4];
      const double rr = wall ? rl : (double)wr[0], pr = wall ? pl : (double)wr[4];
      double irl = frcp(rl), a2l = G.g * pl * irl;
      const double ral = frsq(a2l), al = a2l * ral;
      const K14 KL = make_k14(G, pl, al, irl, ral);
      double ar = al, rar = ral;
      K14 KR = KL;
      if (!wall) {
        double irr = frcp(rr), a2r = G.g * pr * irr;
        rar = frsq(a2r);
        ar = a2r * rar;
        KR = make_k14(G, pr, ar, irr, rar);
      }
      const bool vac = G.two_gm1 * (al + ar) <= (double)unr - (double)unl;
      TR14 tr{};
      double guess = -1.0;  // the two-rarefaction value
      bool gate = false;
      if (!vac) {
        tr = tr14(G, unl, unr, al, ar, KL, KR);
        gate = !wall && tr.p > fmin(KL.p, KR.p);
        guess = tr.p;
      }
      if ((FEAT & 2) && gate && net) {
        info.evaluated = 1;
        if (fabsf(ym) > a.guess_gate) {
          double gm = tr.p * exp((double)ym);
          if (gm > 0.0 && isfinite(gm)) {
            guess = gm;
            info.used = 1;
          } else {
            info.rejected = 1;
          }
        }
      }
      // (with vacuum data the solver returns before it looks at tr)
      Star st = solve_star14(G, unl, unr, al, ar, KL, KR, a.s.newton_tol, a.s.newton_max_iter,
                             guess, &tr);
      info.iters = st.iters;
      info.fallback = st.fallback;
      info.vacuum = st.vacuum;
      if ((FEAT & 1) && !st.vacuum) {
        const int cat = (st.p > fmin(pl, pr) ? 1 : 0) + (st.p > fmax(pl, pr) ? 1 : 0);
        hist_key = 8 * cat + min(max(st.iters, 1), 8) - 1;
        hist_iters = st.iters;
      }
      if (gate) {
        info.gated = 1;
        info.gated_iters = st.iters;
        if ((FEAT & 1) && a.log_cap > 0) {
          unsigned long long h = mix64(a.log_seed ^ mix64(((unsigned long long)r.x << 24) ^ a.subit));
          if ((double)(h >> 11) * 0x1.0p-53 < a.log_rate) {
            unsigned long long slot = atomicAdd(a.log_count, 1ull);
            if (slot < (unsigned long long)a.log_cap) {
              float* row = a.log_rows + 7 * slot;
              face_features<T>(G, wl, wr, unl, unr, x);
              for (int k = 0; k < kMlpIn; ++k) row[k] = x[k];
              row[6] = (float)log(st.p / tr.p);
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
                             (T)ar, (T)KR.ip, (T)rar, (T)st.p, (T)st.u, rs, us, ps, st.zl,
                             st.zr);
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
    store_face_flux(a, r, dt_min, phi, wall, i0, i1, i2);
  }
  if ((FEAT & 1) && a.dnewton) newton_hist_add(a.dnewton, hist_key, hist_iters);
  add_info(acc, info);
}

// One face record: the two face values (or cell states at first order)
// from memory, then flux_feat_w.
template <int ORDER, typename T, int FEAT>
__device__ inline void flux_feat_item(const FluxArgs<T>& a, bool valid, int4 r, double dt_min,
                                      uint16_t* wave_lds, SolveInfo& acc, double& i0,
                                      double& i1, double& i2, bool compact = false) {
  T wl[5] = {1, 0, 0, 0, 1}, wr[5] = {1, 0, 0, 0, 1};
  if (valid) {
    load_side<ORDER, T>(a, r.y, wl, compact);
    if (r.z >= 0) load_side<ORDER, T>(a, r.z, wr, compact);
  }
  flux_feat_w<T, FEAT>(a, valid, r, wl, wr, dt_min, wave_lds, acc, i0, i1, i2);
}

// Adds s_m q_m to acc for the faces m of a cell whose bit is set in act
// (act != 0), in local face order: f the cell's 4 face ids, q_m the face's
// stored flux, s_m = +h_m where the cell is the higher id of the face
// (bit 16 + m of pk), -h_m otherwise; a moving mesh also adds -s_m sF to
// accv.  The fluxes of all the active faces are requested together (an
// inactive slot reads an active face's flux again and adds nothing), so the
// sum waits on one trip to memory rather than one per face.
template <typename T, bool MOVE>
__device__ inline void add_face_fluxes(const int* f, uint32_t pk, unsigned act, const double* h,
                                       const T* __restrict__ Q, const double* __restrict__ sF,
                                       double* acc, double& accv) {
  const int fa = (act & 1u) ? f[0] : (act & 2u) ? f[1] : (act & 4u) ? f[2] : f[3];
  T q[4][5];
  double sv[4];
  for (int m = 0; m < 4; ++m) {
    const int fm = ((act >> m) & 1u) ? f[m] : fa;
    const T* p = Q + 5 * (size_t)fm;
    for (int k = 0; k < 5; ++k) q[m][k] = p[k];
    if (MOVE) sv[m] = sF[fm];
  }
  for (int m = 0; m < 4; ++m) {
    const bool on = (act >> m) & 1u;
    const double sm = (pk & (1u << (16 + m))) ? h[m] : -h[m];
    for (int k = 0; k < 5; ++k) {
      const double a = acc[k] + sm * (double)q[m][k];
      acc[k] = on ? a : acc[k];
    }
    if (MOVE) {
      const double a = accv + (-sm) * sv[m];
      accv = on ? a : accv;
    }
  }
}


// A cell ending its step applies its flux sum acc to its state u0 and
// volume v (both already loaded): U += acc / V on a fixed mesh; on a moving
// mesh its content and volume change together (geometric conservation),
// V' = V + accv, U' = (V U + acc) / V'.  Returns false on a non-finite state
// or a non-positive volume.
// (Vw: the writable volume array of a moving mesh, null otherwise)
template <bool MOVE>
__device__ inline bool apply_cell(int i, const double* acc, double accv, const double* u0,
                                  double v, double* __restrict__ Vw, double* __restrict__ U) {
  bool bad = false;
  if (MOVE) {
    const double vn = v + accv;
    for (int k = 0; k < 5; ++k) {
      const double u = (v * u0[k] + acc[k]) / vn;
      U[5 * (size_t)i + k] = u;
      bad |= !isfinite(u);
    }
    Vw[i] = vn;
    bad |= !(vn > 0.0);
  } else {
    for (int k = 0; k < 5; ++k) {
      const double u = u0[k] + acc[k] / v;
      U[5 * (size_t)i + k] = u;
      bad |= !isfinite(u);
    }
  }
  return !bad;
}

// Gather mode, per cell with an active face or whose step ends: add the
// active faces' time-integrated fluxes q = 2^tau_f dt_min Phi in local face
// order (-q where the cell is the lower id of the face, +q otherwise), then
// U += R / V, R = 0 for ending steps.  A cell with kEarlyBit applies the
// sum of its faces at its step's start instead (its accumulator stays 0).
// Returns false on a non-finite updated state.
template <typename T, bool MOVE = false>
__device__ inline bool cell_gather_item(int i, int nc, const uint32_t* __restrict__ fpack,
                                        const int* __restrict__ c2f,
                                        const T* __restrict__ Q, double dt_min,
                                        const double* __restrict__ vol, double* __restrict__ U,
                                        double* __restrict__ R, int tau_s, int tau_upd,
                                        const double* __restrict__ sF = nullptr,
                                        double* __restrict__ Rv = nullptr,
                                        double* __restrict__ Vw = nullptr) {
  // everything indexed by the cell alone is requested in one trip: the
  // packed word, the face ids, the state and the volume (the last two are
  // read whether or not the cell applies a sum now)
  const uint32_t pk = fpack[i];
  int f[4];
  for (int m = 0; m < 4; ++m) f[m] = c2f[m * nc + i];
  double u0[5];
  for (int k = 0; k < 5; ++k) u0[k] = U[5 * (size_t)i + k];
  const double v0 = MOVE ? Vw[i] : vol[i];
  const int ti = (pk >> 20) & 15;
  double acc[5] = {0, 0, 0, 0, 0};
  double accv = 0.0;  // moving mesh: swept volume, -dt_f sF per face as the flux
  if (pk & kEarlyBit) {
    if (ti > tau_s) return true;  // applied at the step's start
    const double dtf = ldexp(dt_min, ti);
    const double h[4] = {dtf, dtf, dtf, dtf};
    add_face_fluxes<T, MOVE>(f, pk, 0xfu, h, Q, sF, acc, accv);
    return apply_cell<MOVE>(i, acc, accv, u0, v0, Vw, U);
  }
  unsigned act = 0;
  double h[4];
  for (int m = 0; m < 4; ++m) {
    const int tf = (int)((pk >> (4 * m)) & 15);
    h[m] = ldexp(dt_min, tf);
    act |= (unsigned)(tf <= tau_s) << m;
  }
  const bool ends = ti <= tau_upd;
  if (!act && !ends) return true;
  double* Ri = R + 5 * (size_t)i;
  for (int k = 0; k < 5; ++k) acc[k] = Ri[k];
  if (MOVE) accv = Rv[i];
  if (act) add_face_fluxes<T, MOVE>(f, pk, act, h, Q, sF, acc, accv);
  if (ends) {
    for (int k = 0; k < 5; ++k) Ri[k] = 0.0;
    if (MOVE) Rv[i] = 0.0;
    return apply_cell<MOVE>(i, acc, accv, u0, v0, Vw, U);
  }
  for (int k = 0; k < 5; ++k) Ri[k] = acc[k];
  if (MOVE) Rv[i] = accv;
  return true;
}

// ---------------------------------------------------------------------------
// predictor/corrector form of the level steps (Sec. 2.2, Alg. 2: predictor,
// extensive prediction, interpolation of the slower levels, corrector,
// extensive correction).  Per cell: U the state at its step start, D the
// change its predictor forecasts for the step, Ut its state at the time the
// next face pass looks at: U + w D, w the elapsed fraction of its step.

// After the predictor fluxes phi0 of a subiteration are stored, per cell of
// the mesh: a cell whose step starts now (tau <= tau_s) forms
// D = 2^tau dt_min (sum of its faces' +-phi0, local order) / V; then every
// cell's state at the end of the subiteration, unit s of the iteration, is
// written to Ut, with w = (s mod 2^tau) / 2^tau, or 1 where its step ends.
template <typename T>
__device__ inline void predict_item(int i, int nc, const uint32_t* __restrict__ fpack,
                                    const int* __restrict__ c2f, const T* __restrict__ Q0,
                                    double dt_min, const double* __restrict__ vol,
                                    const double* __restrict__ U, double* __restrict__ D,
                                    double* __restrict__ Ut, int tau_s, int s,
                                    const int8_t* __restrict__ nkey, int upd) {
  const uint32_t pk = fpack[i];
  const int ti = (pk >> 20) & 15;
  // the interpolated state at the subiteration's end is read by the
  // corrector pass and the next predictor pass, both over the faces of
  // tau_f <= upd: the cells with such a face and their neighbours (their
  // gradient stencils), nkey <= upd.  A cell whose step does not start and
  // that no such pass reads has nothing to write (it is written again
  // before it is read).
  if (ti > tau_s && nkey[i] > upd) return;
  double d[5];
  double* Di = D + 5 * (size_t)i;
  if (ti <= tau_s) {
    int f[4];
    for (int m = 0; m < 4; ++m) f[m] = c2f[m * nc + i];
    double acc[5] = {0, 0, 0, 0, 0}, accv = 0.0;
    const double one[4] = {1.0, 1.0, 1.0, 1.0};
    add_face_fluxes<T, false>(f, pk, 0xfu, one, Q0, nullptr, acc, accv);
    const double dtc = ldexp(dt_min, ti), v = vol[i];
    for (int k = 0; k < 5; ++k) {
      d[k] = dtc * acc[k] / v;
      Di[k] = d[k];
    }
  } else {
    for (int k = 0; k < 5; ++k) d[k] = Di[k];
  }
  const int per = 1 << ti, r = s & (per - 1);
  const double w = r == 0 ? 1.0 : (double)r / (double)per;
  const double* Ui = U + 5 * (size_t)i;
  double* Uti = Ut + 5 * (size_t)i;
  for (int k = 0; k < 5; ++k) Uti[k] = Ui[k] + w * d[k];
}

// Corrector gather, per cell with a face whose step ends now (tau_f <= upd):
// add those faces' q = 2^tau_f dt_min (phi0 + phi1) / 2 in local face order
// (the corrector pass stored phi0 + phi1);
// a cell whose own step ends applies its sum, U += R / V, and its state for
// the next predictor is the new U.  Returns false on a non-finite state.
template <typename T>
__device__ inline bool cell_gather2_item(int i, int nc, const uint32_t* __restrict__ fpack,
                                         const int* __restrict__ c2f, const T* __restrict__ Q,
                                         double dt_min, const double* __restrict__ vol,
                                         double* __restrict__ U, double* __restrict__ Ut,
                                         double* __restrict__ R, int tau_upd) {
  // the packed word, face ids, accumulator, state and volume in one trip
  const uint32_t pk = fpack[i];
  int f[4];
  for (int m = 0; m < 4; ++m) f[m] = c2f[m * nc + i];
  double* Ri = R + 5 * (size_t)i;
  double acc[5], u0[5], accv = 0.0;
  for (int k = 0; k < 5; ++k) {
    acc[k] = Ri[k];
    u0[k] = U[5 * (size_t)i + k];
  }
  const double v = vol[i];
  const int ti = (pk >> 20) & 15;
  const bool ends = ti <= tau_upd;
  unsigned act = 0;
  double h[4];
  for (int m = 0; m < 4; ++m) {
    const int tf = (int)((pk >> (4 * m)) & 15);
    h[m] = ldexp(dt_min, tf - 1);
    act |= (unsigned)(tf <= tau_upd) << m;
  }
  if (!act && !ends) return true;
  if (act) add_face_fluxes<T, false>(f, pk, act, h, Q, nullptr, acc, accv);
  if (ends) {
    bool bad = false;
    for (int k = 0; k < 5; ++k) {
      const double u = u0[k] + acc[k] / v;
      U[5 * (size_t)i + k] = u;
      Ut[5 * (size_t)i + k] = u;
      Ri[k] = 0.0;
      bad |= !isfinite(u);
    }
    return !bad;
  }
  for (int k = 0; k < 5; ++k) Ri[k] = acc[k];
  return true;
}

}  // namespace tafv
