// Internal data structures of the tafv library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tafv.h"

namespace tafv {

constexpr int kMaxLevels = 8;
constexpr int kMaxColours = 8;
constexpr int kMaxKeys = kMaxColours * kMaxLevels;
// device counters: kCounterSlots slots of kCounterStride 8-byte words
constexpr int kCounterSlots = 64;
constexpr int kCounterStride = 16;
constexpr int kCounterWords = kCounterSlots * kCounterStride;

// Host-side mesh after preprocessing: faces in colour-major order.
struct HostMesh {
  int64_t nc = 0, nf = 0, nbnd = 0;
  int ncolours = 0;
  int64_t colour_start[kMaxColours + 1] = {0};
  // faces
  std::vector<int32_t> fhL, fhR;   // half-face ids 4*cell + slot; fhR = -1 on the boundary
  std::vector<int8_t> fcol;        // colour of each face
  std::vector<double> fA;          // [3][nf] area vector out of the lower cell
  // cells
  std::vector<int32_t> nb;         // [4][nc] neighbour across slot m, or -(face+1)
  std::vector<int32_t> c2f;        // [4][nc] face of slot m
  std::vector<double> lsq;         // [12][nc] least-squares coefficient vectors
  std::vector<double> rf;          // [12][nc] face centroid minus cell centroid
  std::vector<double> vol;         // [nc]
  std::vector<int32_t> perm;       // [nc] internal cell -> caller cell
};

// Builds faces, geometry, colouring and least-squares weights.  Returns
// TAFV_OK or TAFV_E_MESH with a message.
// colour_major: faces ordered by (colour, lower cell, higher cell), else by
// (lower cell, higher cell).  morton: internal cells in Z-order of their
// centroids, else in the caller's order.
tafv_status build_host_mesh(int64_t n_nodes, const double* xyz, int64_t n_tets,
                            const int64_t* tets, bool colour_major, bool morton,
                            HostMesh* out, std::string* err);

// Partition scratch for building level-ordered index lists.
struct Partition {
  int32_t* list = nullptr;     // [n] indices sorted by key, stable
  int32_t* counts = nullptr;   // [kMaxKeys][nblocks]
  int32_t* offs = nullptr;     // [kMaxKeys][nblocks] exclusive scan of counts
  void* scan_tmp = nullptr;    // device scan scratch
  size_t scan_bytes = 0;
  int32_t* start = nullptr;    // [kMaxKeys + 1] device
  int32_t nblocks = 0;
};

// Device state of one mesh.
struct DevMesh {
  int32_t nc = 0, nf = 0, nb = 0, ncolours = 0;
  int32_t max_levels = 5;
  int32_t scatter = TAFV_SCATTER_GATHER;
  int64_t colour_start[kMaxColours + 1] = {0};
  // geometry
  int32_t *fhL = nullptr, *fhR = nullptr;
  int8_t* fcol = nullptr;
  double* fA = nullptr;
  float* fA32 = nullptr;
  int32_t *nb_ = nullptr, *c2f = nullptr;
  double *lsq = nullptr, *rf = nullptr, *vol = nullptr;
  float *lsq32 = nullptr, *rf32 = nullptr;
  // state
  double* U = nullptr;     // [nc][5]
  double* U0 = nullptr;    // [nc][5] state of the last state_init
  double* R = nullptr;     // [nc][5]
  int8_t* lev = nullptr;   // [nc]
  int8_t* lev2 = nullptr;  // [nc]
  double* dt = nullptr;    // [nc]
  void* Wf = nullptr;      // [4][5][nc] reconstructed primitives (double or float)
  double* Q = nullptr;     // [nf][5] gather mode: time-integrated face fluxes
  int4* frec = nullptr;    // [nf] face records {f, hL, hR, tau_f} in partition order
  // schedule lists
  Partition pf, pc;        // faces by (colour, tau_f); cells by tau_g
  int8_t* fkey = nullptr;  // [nf] partition key of each face
  int8_t* ckey = nullptr;  // [nc] tau_g of each cell
  int* chist = nullptr;    // [64] cell count per (tau_g, tau)
  int* rb = nullptr;       // packed readback buffer
  uint32_t* fpack = nullptr; // [nc] per local face m: tau_f in bits 4m..4m+3, the cell
                           // is the higher-id side in bit 16+m; tau in bits 20..23
  int32_t* perm = nullptr; // [nc] internal cell -> caller cell
  double* xfer = nullptr;  // [nc][5] staging for host transfers in caller order
  // device scalars: [0] dt_min bits, [1] theta, [2] non-finite flag
  unsigned long long* dscal = nullptr;
  // device counters: newton updates, fallbacks, vacuum; wall impulse x3
  unsigned long long* dcount = nullptr;
  double* dimpulse = nullptr;
  // host schedule mirror
  bool has_state = false;
  int32_t phase = 0, theta = 0;
  double dt_min = 0.0, t = 0.0;
  int32_t hstart_f[kMaxKeys + 1] = {0};
  int32_t hstart_c[kMaxLevels + 1] = {0};
  int32_t hhist[kMaxKeys] = {0};
  bool classified = false;
  tafv_stats st{};
};

struct ProfileClass {
  const char* name;
  double ms = 0.0;
  int64_t launches = 0, items = 0;
};

}  // namespace tafv

struct tafv_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tafv_params prm{};
  std::vector<tafv::DevMesh*> meshes;
  std::string err;
  // host pinned readback buffer
  int32_t* hpin = nullptr;
  // profiling
  bool profile = false;
  std::vector<tafv::ProfileClass> prof;
  struct PendingEvent { hipEvent_t a, b; int cls; int64_t items; };
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> event_pool;
  // learned guess: FP32 master parameters, Adam moments, device network
  float *mlp_th = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_grad = nullptr;
  float *mlp_gpart = nullptr, *mlp_lpart = nullptr, *mlp_loss = nullptr;
  int64_t mlp_gpart_blocks = 0;
  void* mlp_w = nullptr;  // tafv::MlpDev
  bool mlp_ready = false;
  int mlp_step = 0;
  // face log
  float* log_rows = nullptr;
  unsigned long long* log_count = nullptr;
  int64_t log_cap = 0;
  double log_rate = 0.0;
  uint64_t log_seed = 0;
};
