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
// Newton-update histogram by category: kCounterSlots slots of kNewtonWords
constexpr int kNewtonWords = 32;

// Host-side mesh after preprocessing: faces in colour-major order.
struct HostMesh {
  int64_t nc = 0, nf = 0, nbnd = 0;
  int ncolours = 0;
  int64_t colour_start[kMaxColours + 1] = {0};
  // faces
  std::vector<int32_t> fhL, fhR;   // half-face ids 4*cell + slot; fhR = -1 on the boundary
  std::vector<int8_t> fcol;        // colour of each face
  std::vector<double> fA;          // [3][nf] area vector out of the lower cell
  std::vector<int32_t> fnode;      // [3][nf] the face's node ids, ascending
  int64_t n_nodes = 0;
  // cells
  std::vector<int32_t> nb;         // [4][nc] neighbour across slot m, or -(face+1)
  std::vector<int32_t> c2f;        // [4][nc] face of slot m
  std::vector<double> grc;         // [12][nc] reconstruction coefficients c_j . r_m, m < 3
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
  int32_t* offs = nullptr;     // [kMaxKeys][nblocks] exclusive scan of each key's counts
  int32_t* tot = nullptr;      // [kMaxKeys] count of each key
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
  double *grc = nullptr, *vol = nullptr;
  double* vol0 = nullptr;   // [nc] volumes of the uploaded geometry
  int32_t* fnode = nullptr; // [3][nf] node ids of each face, ascending
  int64_t n_nodes = 0;
  float *grc32 = nullptr;
  // state
  double* U = nullptr;     // [nc][5]
  double* U0 = nullptr;    // [nc][5] state of the last state_init
  double* R = nullptr;     // [nc][5]
  int8_t* lev = nullptr;   // [nc]
  int8_t* lev2 = nullptr;  // [nc] (batched form: ping-pong sweeps)
  unsigned* sweepf = nullptr;  // [kMaxLevels] lowering sweep k changed a level
  double* dt = nullptr;    // [nc]
  void* Wf = nullptr;      // [4][5][nc] reconstructed primitives (double or float)
  void* Q = nullptr;       // [nf][5] gather mode: face fluxes |A| F . n in the flux
                           // precision (double or float); the cells scale them
                           // by 2^tau_f dt_min in FP64
  // moving mesh only: per face the volume rate sF = w_f . A_f it sweeps,
  // per cell the swept volume not yet applied; vol then holds the current
  // cell volumes
  bool moving = false;
  double* sF = nullptr;    // [nf]
  double* Rv = nullptr;    // [nc]
  // predictor/corrector form only (time order 2)
  void* Q0 = nullptr;      // [nf][5] predictor flux of each face's current step (flux
                           // precision)
  double* D = nullptr;     // [nc][5] predicted change of each cell's current step
  double* Ut = nullptr;    // [nc][5] cell states at the time the next face pass reads
  int4* frec = nullptr;    // [nf] face records {f, hL, hR, tau_f} in partition order
  // gather mode, second order: faces whose fluxes the whole-mesh gradient
  // launch computes (both sides, or the one side of a boundary face, in one
  // chunk of kFuseChunk cells): flocal[f] = 1 for them, and per chunk their
  // list (see LocalFaces).  While split_local is set (chosen at each
  // classification: the fused launches can run), the face list is sorted by
  // tau_f + 8 flocal, the faces between chunks first.
  // pipelined whole-mesh subiterations: chunk k holds cells
  // [pipe_c[k], pipe_c[k + 1]) and the faces [pipe_f[k], pipe_f[k + 1])
  // whose first (lower) cell lies in it; pipe_k = 1: no pipeline
  int pipe_k = 1;
  std::vector<int32_t> pipe_c, pipe_f;
  int8_t* flocal = nullptr;  // [nf]
  int32_t* lf_start = nullptr;  // [chunks + 1]
  int2* lf_face = nullptr;      // [n_local]
  int32_t n_local = 0;
  bool split_local = false;
  // While split_local is set, the face values of the half-faces whose
  // neighbour lies in another chunk go to a compact array Wx [nx][5] in
  // cell order (cell c's from xb[c], by slot), and the face records of the
  // faces between chunks take their positions there (fxL, fxR; the other
  // faces keep their half-face ids).
  void* Wx = nullptr;
  int32_t* xb = nullptr;   // [nc]
  int32_t* fxL = nullptr;  // [nf]
  int32_t* fxR = nullptr;  // [nf]
  int64_t nx = 0;
  // schedule lists
  Partition pf, pc, pg;    // faces by (colour, tau_f); cells by tau_g; the gather's
                           // cell list (see cells_gather)
  int8_t* fkey = nullptr;  // [nf] partition key of each face
  int8_t* ckey = nullptr;  // [nc] tau_g of each cell
  // [nc] predictor/corrector form: the smallest tau_g over the cell and its
  // face neighbours (which face passes read its interpolated state)
  int8_t* nkey = nullptr;
  unsigned long long* dnewton = nullptr;  // [kCounterSlots][kNewtonWords]
  int8_t* lkey = nullptr;  // [nc] key of the gather's cell list (see list_cell)
  int* chist = nullptr;    // [kCounterSlots][64] cell count per (tau_g, tau), summed
                           // over the slots by the readback kernel
  int* rb = nullptr;       // packed readback buffer
  uint32_t* fpack = nullptr; // [nc] per local face m: tau_f in bits 4m..4m+3, the cell
                           // is the higher-id side in bit 16+m; tau in bits 20..23
  int32_t* perm = nullptr; // [nc] internal cell -> caller cell
  double* xfer = nullptr;  // [nc][5] staging for host transfers in caller order
  // device scalars: [0] dt_min bits, [1] theta, [2] non-finite flag
  unsigned long long* dscal = nullptr;
  // per-block minima of dt (bits), spread over kCounterSlots slots
  unsigned long long* dmin = nullptr;
  // device counters: newton updates, fallbacks, vacuum; wall impulse x3
  unsigned long long* dcount = nullptr;
  double* dimpulse = nullptr;
  // host schedule mirror
  bool has_state = false;
  int32_t phase = 0, theta = 0;
  double dt_min = 0.0, t = 0.0;
  int32_t hstart_f[kMaxKeys + 1] = {0};
  int32_t hstart_c[kMaxLevels + 1] = {0};
  int32_t hstart_g[2 * kMaxLevels + 1] = {0};  // starts of the gather list's keys
  int32_t hhist[kMaxKeys] = {0};
  bool classified = false;
  tafv_stats st{};
};

// Per-mesh schedule of the batched form, resident on the device: the
// segment of the merged arrays, the level cap, Alg. 2's schedule state and
// the per-subiteration work counts.
struct BatchSched {
  int32_t c0, nc, f0, nf;             // cells [c0, c0 + nc), faces [f0, f0 + nf)
  int32_t L, theta, phase, classified;
  int32_t reclass, tau_s, upd, n_grad; // this subiteration: classify?, levels, work
  int32_t n_flux, n_gather, pad0, pad1;
  double dt_min, t;
  unsigned long long dtbits;          // running minimum of dt (bit pattern)
  int64_t subiterations, cell_updates, face_solves;
  int64_t cells_per_level[kMaxLevels];
  int32_t fstart[kMaxLevels + 1];     // face list: start of tau_f = k (global position)
  int32_t cstart[kMaxLevels + 1];     // cell list: start of tau_g = k
  int32_t hist[kMaxKeys];             // cells per (tau_g, tau)
};

// Launch settings of one work class of the batched kernels.
struct LaunchSet {
  int32_t grid = 0;  // blocks of the persistent launch
  int32_t grab = 1;  // consecutive unit groups a block takes at a time; 0: one
                     // group per block, grid = the static count of groups
  int32_t bs = 256;  // threads per block (64, 128, 256 or 512)
};

struct DevMesh;
struct HostMesh;

// Batched form: the uploaded meshes merged into one set of arrays (cell,
// face and half-face ids offset per mesh), with a schedule per mesh.
struct Batch {
  std::vector<HostMesh*> hosts;       // uploaded, merged at the first use
  std::vector<int32_t> L;
  std::vector<uint8_t> has_state;
  bool built = false;
  int32_t nmesh = 0;
  DevMesh* m = nullptr;
  BatchSched* dsched = nullptr;
  std::vector<BatchSched> hsched;     // host copy after each call
  // static tile prefixes [nmesh + 1]: cell tiles and face tiles of kBlock
  // items, cell chunks and face chunks of the partitions
  int32_t *ct = nullptr, *ft = nullptr, *cc = nullptr, *fc = nullptr;
  int32_t n_cc = 0, n_fc = 0, n_ft = 0, n_ct = 0, n_cu = 0, n_fu = 0;
  int32_t *cnt_f = nullptr, *cnt_c = nullptr;  // [8 * chunks] counts, then offsets
  int32_t* tp = nullptr;              // [3][nmesh + 1] tiles: gradient, flux, cells
  int32_t* rp = nullptr;              // [4][nmesh + 1] reclassification tiles and chunks
  double* tmin = nullptr;             // [cell tiles] per-tile minimum of dt
  int* thist = nullptr;               // [cell tiles][64] per-tile level histogram
  int32_t lmax = 1;
  LaunchSet set[3];                   // gradient, flux (fixed: one tile per
                                      // block over all face tiles), cells
  int32_t tuned = 0;                  // 0 defaults, 1 timed here, 2 read from the cache
  int32_t graph = 1, autotune = 1;
  std::string cache;
  hipStream_t cap = nullptr;          // capture stream
  std::vector<std::pair<int64_t, hipGraphExec_t>> execs;
  int64_t exec_key = -1;
  tafv_stats last{};                  // cumulative slot counters at the last call
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
  // host pinned readback buffer, and the event that marks the readback's copy
  int32_t* hpin = nullptr;
  hipEvent_t rb_event = nullptr;
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
  // batched form (params.batch = 1)
  tafv::Batch* batch = nullptr;
  // device memory: the caller's allocator (tafv_set_allocator) or, when
  // none is set, hipMalloc / hipFree; live_buffers counts what the context
  // holds, so the allocator can only change while it holds nothing
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*dealloc_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  int64_t live_buffers = 0;
};

namespace tafv {

// shared by the C-ABI and the batched driver (capi.hip)
tafv_status set_error(tafv_ctx* c, tafv_status st, const std::string& msg);
tafv_status hip_error(tafv_ctx* c, hipError_t e, const char* what);
tafv_status upload_host_mesh(tafv_ctx* c, const HostMesh& hm, DevMesh** out);
void free_dev_mesh(tafv_ctx* c, DevMesh* m);
// every device buffer of a context goes through these two; dev_malloc
// returns hipErrorOutOfMemory when the allocator returns NULL
hipError_t dev_malloc(tafv_ctx* c, void** p, size_t bytes);
void dev_free(tafv_ctx* c, void* p);
template <typename T>
hipError_t dev_alloc(tafv_ctx* c, T** p, size_t bytes) {
  return dev_malloc(c, reinterpret_cast<void**>(p), bytes);
}
// sums the slot counters of m into st (newton ... guess_used, wall impulse)
tafv_status read_slot_counters(tafv_ctx* c, DevMesh& m, tafv_stats* st);

// per-kernel-class timing with HIP events on the context stream
enum { P_CLASSIFY = 0, P_GRAD = 1, P_FLUX = 2, P_UPDATE = 3, P_GATHER = 4, P_PREDICT = 5,
       P_FLUX_CORR = 6, P_GRAD_FLUX = 7, P_N = 8 };
struct ProfScope {
  tafv_ctx* c;
  int cls;
  int64_t items;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(tafv_ctx* c_, int cls_, int64_t items_) : c(c_), cls(cls_), items(items_) {
    if (!c || !c->profile) return;
    a = take();
    b = take();
    (void)hipEventRecord(a, c->stream);
  }
  ~ProfScope() {
    if (!c || !c->profile) return;
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({a, b, cls, items});
  }
  hipEvent_t take() {
    if (!c->event_pool.empty()) {
      hipEvent_t e = c->event_pool.back();
      c->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

// batched driver (batch.hip)
tafv_status batch_upload(tafv_ctx* c, HostMesh* hm, int32_t* mesh_id);
tafv_status batch_mesh_params(tafv_ctx* c, int32_t mesh_id, int32_t max_levels);
tafv_status batch_state_init(tafv_ctx* c, int32_t mesh_id, const double* prim);
tafv_status batch_state_reset(tafv_ctx* c, int32_t mesh_id);
tafv_status batch_advance(tafv_ctx* c, int64_t n, tafv_stats* out);
tafv_status batch_mesh_stats(tafv_ctx* c, int32_t mesh_id, tafv_stats* out);
tafv_status batch_state_read(tafv_ctx* c, int32_t mesh_id, double* cons, int8_t* levels);
tafv_status batch_checkpoint_read(tafv_ctx* c, int32_t mesh_id, double* cons, double* accum,
                                  int8_t* levels, int32_t* phase, int32_t* theta,
                                  double* dt_min, double* t);
tafv_status batch_config(tafv_ctx* c, int32_t graph, int32_t autotune, const char* cache);
tafv_status batch_info(tafv_ctx* c, int32_t* info, int32_t n);
void batch_invalidate(tafv_ctx* c);
void batch_free(tafv_ctx* c);

}  // namespace tafv
