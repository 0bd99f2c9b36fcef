// C-ABI of the tafv library: context, mesh upload, state, the subiteration
// driver of Alg. 2 (Sec. 2.2), checkpoints, counters and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "mlp_kernels.h"
#include "tafv_internal.h"

using namespace tafv;

namespace {

// ---- scratch of the network gradient that allocates nothing ---------------
// tafv_mlp_grad_noalloc keeps its staging and partial results in one
// file-scope device array per GPU instead of buffers it allocates.  Layout
// (floats, each part 64-float aligned): per-block partial gradients
// [rows / 64][1313], per-block partial losses [rows / 64], inputs x
// [rows][6], targets [rows], the gradient [1313], the loss [1].
constexpr int64_t kScrRows = TAFV_MLP_GRAD_NOALLOC_MAX_ROWS;
constexpr int64_t kScrBlocks = kScrRows / 64;
constexpr size_t scr_up(size_t n) { return (n + 63) / 64 * 64; }
constexpr size_t kScrGpart = 0;
constexpr size_t kScrLpart = scr_up(kScrGpart + (size_t)kScrBlocks * kMlpParams);
constexpr size_t kScrX = scr_up(kScrLpart + kScrBlocks);
constexpr size_t kScrT = scr_up(kScrX + (size_t)kScrRows * kMlpIn);
constexpr size_t kScrGrad = scr_up(kScrT + kScrRows);
constexpr size_t kScrLoss = scr_up(kScrGrad + kMlpParams);
constexpr size_t kScrFloats = scr_up(kScrLoss + 1);
static_assert(kScrRows % 64 == 0, "whole 64-row blocks");

static __device__ __align__(256) float scratch[kScrFloats];

// The array's device address on each GPU, taken once per device at context
// creation (the host-side name is not a device address).
constexpr int kScrMaxDevices = 64;
std::mutex g_scr_mu;
float* g_scr_ptr[kScrMaxDevices] = {};

// with `device` current
hipError_t scratch_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scr_mu);
  if (device < 0 || device >= kScrMaxDevices) return hipErrorInvalidDevice;
  if (g_scr_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scr_ptr[device] = static_cast<float*>(p);
  return hipSuccess;
}

float* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scr_mu);
  return (device >= 0 && device < kScrMaxDevices) ? g_scr_ptr[device] : nullptr;
}

// per-kernel timing classes; "flux_corrector" is the corrector pass of the
// predictor/corrector form (it also reads the predictor flux), "grad_flux"
// the gradient launches that also compute the faces local to a chunk (items:
// cells)
const char* kProfNames[] = {"classify", "grad",    "flux",           "update",
                            "gather",   "predict", "flux_corrector", "grad_flux"};

thread_local std::string g_create_err;

tafv_status fail(tafv_ctx* c, tafv_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return st;
}

tafv_status hip_fail(tafv_ctx* c, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? TAFV_E_OOM : TAFV_E_DEVICE, msg);
}

#define HIP_TRY(c, expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail((c), e_, #expr); \
  } while (0)

template <typename T>
hipError_t dalloc(tafv_ctx* c, T** p, size_t n) {
  return dev_malloc(c, (void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

void free_mesh(tafv_ctx* c, DevMesh* m) {
  if (!m) return;
  void* ptrs[] = {m->fhL, m->fhR, m->fcol, m->fA, m->fA32, m->nb_, m->c2f, m->grc,
                  m->vol, m->grc32, m->U, m->U0, m->R, m->lev, m->lev2, m->dt, m->Wf,
                  m->pf.list, m->pf.counts, m->pf.start, m->pc.list, m->pc.counts,
                  m->pc.start, m->dscal, m->dcount, m->dimpulse, m->pf.offs, m->pc.offs,
                  m->pf.tot, m->pc.tot, m->Q, m->frec, m->fkey, m->ckey, m->fpack,
                  m->perm, m->xfer, m->chist, m->rb, m->dmin, m->Q0, m->D, m->Ut, m->nkey,
                  m->vol0, m->fnode, m->sF, m->Rv, m->sweepf, m->lkey, m->pg.list,
                  m->pg.counts, m->pg.start, m->pg.offs, m->pg.tot, m->flocal,
                  m->lf_start, m->lf_face, m->Wx, m->xb, m->fxL, m->fxR, m->dnewton};
  for (void* p : ptrs) dev_free(c, p);
  delete m;
}

StepArgs step_args(const tafv_ctx* c, const DevMesh& m) {
  StepArgs a;
  a.gas = make_gas(c->prm.gamma);
  a.cfl = c->prm.cfl;
  a.newton_tol = c->prm.newton_tol;
  a.level_margin = c->prm.level_margin;
  a.dt_min = m.dt_min;
  a.newton_max_iter = c->prm.newton_max_iter;
  a.boundary = c->prm.boundary;
  a.max_levels = m.max_levels;
  a.precision = c->prm.precision;
  a.order = c->prm.order;
  return a;
}

// level computed in subiteration s = 1..2^theta (Alg. 2): the largest
// tau <= theta with 2^tau dividing s - 1 (theta itself for s = 1)
int subiteration_level(int64_t s, int theta) {
  if (s == 1) return theta;
  int t = 0;
  int64_t x = s - 1;
  while (!(x & 1) && t < theta) {
    x >>= 1;
    ++t;
  }
  return t;
}

// ---- classification at an iteration start ------------------------------

// per-level cell counts of the latest classification; returns theta
int level_histogram(DevMesh& m) {
  int theta = 0;
  for (int t = 0; t < kMaxLevels; ++t) {
    int64_t n = 0;
    for (int g = 0; g < kMaxLevels; ++g) n += m.hhist[g * kMaxLevels + t];
    m.st.cells_per_level[t] = n;
    if (n > 0) theta = t;
  }
  return theta;
}

// moving mesh: a new or reset state starts from the uploaded geometry's
// volumes, with no swept volume pending (the motion itself is kept)
hipError_t reset_volumes(tafv_ctx* c, DevMesh& m) {
  if (!m.moving) return hipSuccess;
  hipError_t e = hipMemcpyAsync(m.vol, m.vol0, sizeof(double) * m.nc, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e == hipSuccess) e = launch_fill_f64(c->stream, m.Rv, 0.0, m.nc);
  return e;
}

// predictor/corrector form: at an iteration start every cell starts a step,
// so its state for the first predictor is U itself
hipError_t sync_time_states(tafv_ctx* c, DevMesh& m) {
  if (!m.Ut) return hipSuccess;
  hipError_t e = hipMemcpyAsync(m.Ut, m.U, sizeof(double) * 5 * m.nc, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e == hipSuccess) e = launch_fill_f64(c->stream, m.D, 0.0, (int64_t)5 * m.nc);
  return e;
}

// cells applying their fluxes at their step's start: gather mode with one
// face pass per step (the spatial order decides which neighbours matter)
int early_order(const tafv_ctx* c, const DevMesh& m) {
  return (m.scatter == TAFV_SCATTER_GATHER && c->prm.time_order == 1) ? c->prm.order : 0;
}

FluxFeatures flux_features(tafv_ctx* c, DevMesh& m);
bool fusable(const tafv_ctx* c, const DevMesh& m, const FluxFeatures& ft);

// Enqueues the classification at an iteration start (time steps, levels,
// sweeps, keys, lists) and the copy of its results to the pinned host
// buffer; c->rb_event marks the copy's end.
tafv_status classify_enqueue(tafv_ctx* c, DevMesh& m) {
  StepArgs a = step_args(c, m);
  m.split_local = fusable(c, m, flux_features(c, m));
  {
    ProfScope ps(c, P_CLASSIFY, m.nc);
    HIP_TRY(c, launch_dt(c->stream, m, a));
    HIP_TRY(c, launch_classify(c->stream, m, a));
    HIP_TRY(c, launch_partitions(c->stream, m, early_order(c, m)));
  }
  // dt_min, flag, list starts, histogram (packed by the partitions)
  HIP_TRY(c, hipMemcpyAsync(c->hpin, m.rb, kReadbackInts * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipEventRecord(c->rb_event, c->stream));
  return TAFV_OK;
}

// Waits for the readback of classify_enqueue and takes over dt_min, theta,
// the list starts and the level histogram.
tafv_status classify_finish(tafv_ctx* c, DevMesh& m) {
  HIP_TRY(c, hipEventSynchronize(c->rb_event));
  const int K = face_list_keys(m);
  const int32_t* h = c->hpin;
  unsigned long long bits[3];
  std::memcpy(bits, h, sizeof(bits));
  if (bits[2]) return fail(c, TAFV_E_NUMERIC, "non-finite or non-physical cell state");
  double dtmin;
  std::memcpy(&dtmin, &bits[0], sizeof(double));
  if (!(dtmin > 0.0) || !std::isfinite(dtmin))
    return fail(c, TAFV_E_NUMERIC, "no valid time step");
  m.dt_min = dtmin;
  std::memcpy(m.hstart_f, h + kRbFace, (K + 1) * sizeof(int32_t));
  std::memcpy(m.hstart_c, h + kRbCell, (kMaxLevels + 1) * sizeof(int32_t));
  std::memcpy(m.hstart_g, h + kRbGather, (kCellKeys + 1) * sizeof(int32_t));
  std::memcpy(m.hhist, h + kRbHist, kMaxKeys * sizeof(int32_t));
  int theta = level_histogram(m);
  m.theta = theta;
  m.classified = true;
  return TAFV_OK;
}

// cells with an active face when levels <= g start a step (tau_g <= g):
// a prefix of the list sorted by tau_g
CellRange cells_active(const DevMesh& m, int g) {
  CellRange r;
  r.n1 = m.hstart_c[g + 1];
  return r;
}

// The gather's cells, from its own list sorted by 2 k + b (k = the level of
// a cell that applies its fluxes at its step's start, b = 0; k = tau_g of
// the others, b = 1): the cells with an active face (keys up to 2 tau_s + 1)
// and the accumulating cells whose step ends (tau <= upd, so tau_g <= upd:
// keys 2 k + 1 for tau_s < k <= upd); a cell that applies at its step's
// start has nothing left at its end.
ListRanges cells_gather(const DevMesh& m, int tau_s, int upd) {
  ListRanges r;
  r.add(0, m.hstart_g[2 * tau_s + 2]);
  for (int k = tau_s + 1; k <= upd; ++k) r.add(m.hstart_g[2 * k + 1], m.hstart_g[2 * k + 2]);
  return r;
}

// cells with tau <= t
int64_t cells_upto_tau(const DevMesh& m, int t) {
  int64_t n = 0;
  for (int g = 0; g < kMaxLevels; ++g)
    for (int u = 0; u <= t; ++u) n += m.hhist[g * kMaxLevels + u];
  return n;
}

// The active faces of levels <= t (gather mode): a prefix of the face list,
// and, when the faces local to a chunk are listed after the others, the
// prefix of those too.
struct FaceRanges {
  int first1 = 0, n1 = 0, first2 = 0, n2 = 0;
  int count() const { return n1 + n2; }
};
FaceRanges faces_active(const DevMesh& m, int t, bool with_local = true) {
  FaceRanges r;
  r.n1 = m.hstart_f[t + 1];
  if (m.split_local && with_local) {
    r.first2 = m.hstart_f[kMaxLevels];
    r.n2 = m.hstart_f[kMaxLevels + t + 1] - r.first2;
  }
  return r;
}

FluxFeatures flux_features(tafv_ctx* c, DevMesh& m) {
  FluxFeatures ft;
  bool mlp = c->prm.guess == TAFV_GUESS_MLP;
  bool stats = c->prm.guess_stats || c->log_cap > 0;
  ft.feat = (stats ? 1 : 0) | (mlp ? 2 : 0);
  ft.mlp = (const MlpDev*)c->mlp_w;
  ft.log_rows = c->log_rows;
  ft.log_count = c->log_count;
  ft.log_cap = c->log_cap;
  ft.log_rate = c->log_rate;
  ft.log_seed = c->log_seed;
  ft.subit = (unsigned long long)m.st.subiterations;
  ft.guess_gate = (float)c->prm.guess_gate;
  ft.guess_strength = (float)c->prm.guess_strength;
  return ft;
}

// Predictor/corrector form of one subiteration (gather mode).  The cells and
// faces of levels <= tau_s start a step at its beginning, those of levels
// <= upd end one at its end.  Predictor: gradients and fluxes Q0 of the
// starting faces from the states Ut at the beginning; predictions D of the
// starting cells and the states Ut at the end.  Corrector: gradients and
// fluxes of the ending faces from those states, stored as Q = Q0 + phi1;
// sums q = dt_f Q / 2 in the cells; ending cells apply theirs.  The wall
// impulse is the corrector pass's q of each wall face.
tafv_status subiteration2(tafv_ctx* c, DevMesh& m, const StepArgs& a, int tau_s, int upd,
                          int64_t s, int64_t& faces) {
  const double dt_min = m.dt_min;
  const FaceRanges pr = faces_active(m, tau_s), cr = faces_active(m, upd);
  const int pcnt = pr.count(), ccnt = cr.count();
  if (c->prm.order == 2) {
    const CellRange r = cells_active(m, tau_s);
    ProfScope ps(c, P_GRAD, r.count());
    HIP_TRY(c, launch_grad(c->stream, m, a, r, tau_s, m.Ut));
  }
  {
    ProfScope ps(c, P_FLUX, pcnt);
    HIP_TRY(c, launch_flux(c->stream, m, a, 0, pr.n1, flux_features(c, m), m.Ut, m.Q0, 1, nullptr,
                           false, pr.first2, pr.n2, tau_s));
  }
  {
    ProfScope ps(c, P_PREDICT, m.nc);
    HIP_TRY(c, launch_predict(c->stream, m, tau_s, (int)s, upd, dt_min, c->prm.precision));
  }
  if (c->prm.order == 2) {
    const CellRange r = cells_active(m, upd);
    ProfScope ps(c, P_GRAD, r.count());
    HIP_TRY(c, launch_grad(c->stream, m, a, r, upd, m.Ut));
  }
  {
    ProfScope ps(c, P_FLUX_CORR, ccnt);
    HIP_TRY(c, launch_flux(c->stream, m, a, 0, cr.n1, flux_features(c, m), m.Ut, m.Q, 2, m.Q0,
                           false, cr.first2, cr.n2, upd));
  }
  {
    const CellRange r = cells_active(m, upd);
    ProfScope ps(c, P_GATHER, r.count());
    HIP_TRY(c, launch_cell_gather2(c->stream, m, r, upd, dt_min, c->prm.precision));
  }
  faces = (int64_t)pcnt + ccnt;
  return TAFV_OK;
}

// Host bookkeeping at the end of subiteration s (counters, phase, time).
void end_subiteration(DevMesh& m, tafv_stats* acc, int64_t s, int64_t ucnt, int64_t faces) {
  m.phase = (int32_t)(s % ((int64_t)1 << m.theta));
  m.t += m.dt_min;
  m.st.subiterations++;
  m.st.cell_updates += ucnt;
  m.st.face_solves += faces;
  if (acc) {
    acc->subiterations++;
    acc->cell_updates += ucnt;
    acc->face_solves += faces;
  }
}

// Gather mode, second order, forward Euler level steps on a fixed mesh,
// with no flux feature or the learned guess alone (gamma 1.4): a gradient
// launch over the whole mesh can also compute the faces local to a chunk
// (k_grad_flux).  Face statistics and logging keep the flux kernel.
bool fusable(const tafv_ctx* c, const DevMesh& m, const FluxFeatures& ft) {
  const bool feat_ok = ft.feat == 0 || (ft.feat == 2 && c->prm.gamma == 1.4);
  return m.flocal && c->prm.fuse_faces && c->prm.order == 2 && c->prm.time_order == 1 &&
         !m.moving && feat_ok;
}

// A whole-mesh gradient launch computes the chunk-local faces when the
// face list of this iteration keeps them apart.
bool fuse_local_faces(const tafv_ctx* c, const DevMesh& m, const FluxFeatures& ft,
                      int64_t grad_cells) {
  return m.split_local && fusable(c, m, ft) && grad_whole_mesh(m, grad_cells);
}

// Gather mode, second order, forward Euler level steps on a fixed mesh
// whose faces fit its chunks: a subiteration whose gradient and flux
// launches would both cover the whole mesh runs them, with the gather, as
// a pipeline over the chunks.
bool pipelined(const tafv_ctx* c, const DevMesh& m, int64_t grad_cells, int64_t faces) {
  return m.pipe_k > 1 && !m.split_local && !m.moving && c->prm.order == 2 &&
         c->prm.time_order == 1 && m.scatter == TAFV_SCATTER_GATHER &&
         grad_whole_mesh(m, grad_cells) && faces_whole_mesh(m, faces);
}

// Step j of the pipeline: gradients of chunk j, fluxes of chunk j - 1's
// faces (which need the gradients of chunks j - 1 and j), gather of chunk
// j - 2 (whose faces are all computed by then; the gradients that read its
// states are done).  The items of each class go with its first launch.
tafv_status run_pipeline(tafv_ctx* c, DevMesh& m, const StepArgs& a, const FluxFeatures& ft,
                         int tau_s, int upd, double dt_min, bool dt_min_on_device,
                         int64_t grad_cells, int64_t faces, int64_t gather_cells) {
  const int K = m.pipe_k;
  for (int j = 0; j < K + 2; ++j) {
    if (j < K) {
      ProfScope ps(c, P_GRAD, j == 0 ? grad_cells : 0);
      HIP_TRY(c, launch_grad_chunk(c->stream, m, a, tau_s, m.pipe_c[j], m.pipe_c[j + 1]));
    }
    const int k = j - 1;
    if (k >= 0 && k < K) {
      ProfScope ps(c, P_FLUX, k == 0 ? faces : 0);
      HIP_TRY(c, launch_flux_chunk(c->stream, m, a, ft, tau_s, m.pipe_f[k], m.pipe_f[k + 1],
                                   dt_min_on_device));
    }
    const int g = j - 2;
    if (g >= 0 && g < K) {
      ProfScope ps(c, P_GATHER, g == 0 ? gather_cells : 0);
      HIP_TRY(c, launch_gather_chunk(c->stream, m, tau_s, upd, dt_min, c->prm.precision,
                                     m.pipe_c[g], m.pipe_c[g + 1], dt_min_on_device));
    }
  }
  return TAFV_OK;
}

// Gather mode with one face pass per level step on a fixed mesh: the first
// subiteration of an iteration runs at tau_s = theta, so every face and
// every cell take part, and cells of level 0 end their step.  Its launches
// need neither theta nor the list starts (they cover the whole lists, with
// the levels compared against the largest one), and its kernels read dt_min
// on the device; so they are enqueued behind the classification before the
// host waits for its readback, and the GPU computes while the host reads.
bool first_subiteration_ahead(const tafv_ctx* c, const DevMesh& m) {
  return m.scatter == TAFV_SCATTER_GATHER && c->prm.time_order == 1 && !m.moving;
}

tafv_status first_subiteration(tafv_ctx* c, DevMesh& m, tafv_stats* acc) {
  StepArgs a = step_args(c, m);
  const int all = kMaxLevels - 1;  // at least theta
  const FluxFeatures ft = flux_features(c, m);
  const bool fuse = fuse_local_faces(c, m, ft, m.nc);
  if (pipelined(c, m, m.nc, m.nf)) {
    tafv_status st = run_pipeline(c, m, a, ft, all, 0, 0.0, true, m.nc, m.nf, m.nc);
    if (st != TAFV_OK) return st;
    st = classify_finish(c, m);
    if (st != TAFV_OK) return st;
    end_subiteration(m, acc, 1, cells_upto_tau(m, 0), m.nf);
    return TAFV_OK;
  }
  if (c->prm.order == 2) {
    ProfScope ps(c, fuse ? P_GRAD_FLUX : P_GRAD, m.nc);
    if (fuse) {
      HIP_TRY(c, launch_grad_flux(c->stream, m, a, all, ft, true));
    } else {
      CellRange r;
      r.n1 = m.nc;
      HIP_TRY(c, launch_grad(c->stream, m, a, r, all));
    }
  }
  {
    // with the chunk-local faces kept apart, the faces between chunks come
    // first in the face list (the first range); the others follow
    const int n1 = m.split_local ? m.nf - m.n_local : m.nf;
    const int n2 = (m.split_local && !fuse) ? m.n_local : 0;
    ProfScope ps(c, P_FLUX, n1 + n2);
    HIP_TRY(c, launch_flux(c->stream, m, a, 0, n1, ft, nullptr, nullptr, 0, nullptr, true, n1,
                           n2, all));
  }
  {
    ListRanges r;
    r.add(0, m.nc);
    ProfScope ps(c, P_GATHER, m.nc);
    HIP_TRY(c, launch_cell_gather(c->stream, m, r, all, 0, 0.0, c->prm.precision, true));
  }
  tafv_status st = classify_finish(c, m);
  if (st != TAFV_OK) return st;
  end_subiteration(m, acc, 1, cells_upto_tau(m, 0), m.nf);
  return TAFV_OK;
}

tafv_status subiteration(tafv_ctx* c, DevMesh& m, tafv_stats* acc) {
  if (m.phase == 0 && (c->prm.reclassify || !m.classified)) {
    tafv_status st = classify_enqueue(c, m);
    if (st != TAFV_OK) return st;
    if (first_subiteration_ahead(c, m)) return first_subiteration(c, m, acc);
    st = classify_finish(c, m);
    if (st != TAFV_OK) return st;
  }
  StepArgs a = step_args(c, m);
  int tau_s = subiteration_level((int64_t)m.phase + 1, m.theta);
  const FluxFeatures ft = flux_features(c, m);
  int64_t s = (int64_t)m.phase + 1;
  // cells whose step ends after this subiteration: tau_i <= min(theta, ctz(s))
  int upd = 0;
  {
    int64_t x = s;
    while (!(x & 1) && upd < m.theta) {
      x >>= 1;
      ++upd;
    }
  }
  if (c->prm.time_order == 1 && m.scatter == TAFV_SCATTER_GATHER) {
    const int64_t gc = cells_active(m, tau_s).count(), fc = faces_active(m, tau_s).count();
    if (pipelined(c, m, gc, fc)) {
      tafv_status st = run_pipeline(c, m, a, ft, tau_s, upd, m.dt_min, false, gc, fc,
                                    cells_gather(m, tau_s, upd).count());
      if (st != TAFV_OK) return st;
      end_subiteration(m, acc, s, cells_upto_tau(m, upd), fc);
      return TAFV_OK;
    }
  }
  bool fuse = false;
  if (c->prm.order == 2 && c->prm.time_order == 1) {
    const CellRange r = cells_active(m, tau_s);
    fuse = m.scatter == TAFV_SCATTER_GATHER && fuse_local_faces(c, m, ft, r.count());
    ProfScope ps(c, fuse ? P_GRAD_FLUX : P_GRAD, r.count());
    if (fuse) HIP_TRY(c, launch_grad_flux(c->stream, m, a, tau_s, ft, false));
    else HIP_TRY(c, launch_grad(c->stream, m, a, r, tau_s));
  }
  int64_t ucnt = cells_upto_tau(m, upd);
  int64_t faces = 0;
  if (c->prm.time_order == 2) {
    tafv_status st = subiteration2(c, m, a, tau_s, upd, s, faces);
    if (st != TAFV_OK) return st;
  } else if (m.scatter == TAFV_SCATTER_COLOUR) {
    for (int col = 0; col < m.ncolours; ++col) {
      int first = m.hstart_f[col * kMaxLevels];
      int cnt = m.hstart_f[col * kMaxLevels + tau_s + 1] - first;
      faces += cnt;
      ProfScope ps(c, P_FLUX, cnt);
      HIP_TRY(c, launch_flux(c->stream, m, a, first, cnt, FluxFeatures{}));
    }
    const CellRange r = cells_active(m, upd);
    ProfScope ps(c, P_UPDATE, r.count());
    HIP_TRY(c, launch_update(c->stream, m, r, upd));
  } else {
    // with the faces local to a chunk computed by the gradient launch, the
    // flux kernel takes the others
    const FaceRanges fr = faces_active(m, tau_s, !fuse);
    faces = faces_active(m, tau_s).count();
    {
      ProfScope ps(c, P_FLUX, fr.count());
      HIP_TRY(c, launch_flux(c->stream, m, a, 0, fr.n1, ft, nullptr, nullptr, 0, nullptr, false,
                             fr.first2, fr.n2, tau_s));
    }
    const ListRanges r = cells_gather(m, tau_s, upd);
    ProfScope ps(c, P_GATHER, r.count());
    HIP_TRY(c, launch_cell_gather(c->stream, m, r, tau_s, upd, m.dt_min, c->prm.precision));
  }
  end_subiteration(m, acc, s, ucnt, faces);
  return TAFV_OK;
}

tafv_status read_counters(tafv_ctx* c, DevMesh& m) {
  tafv_status st = read_slot_counters(c, m, &m.st);
  if (st != TAFV_OK) return st;
  m.st.theta = m.theta;
  m.st.phase = m.phase;
  m.st.dt_min = m.dt_min;
  m.st.t_reached = m.t;
  return TAFV_OK;
}

bool any_moving(const tafv_ctx* c) {
  for (const DevMesh* m : c->meshes)
    if (m->moving) return true;
  return false;
}

DevMesh* get_mesh(tafv_ctx* c, int32_t id) {
  if (!c || id < 0 || id >= (int32_t)c->meshes.size()) return nullptr;
  return c->meshes[id];
}

}  // namespace

namespace tafv {

tafv_status set_error(tafv_ctx* c, tafv_status st, const std::string& msg) {
  return fail(c, st, msg);
}

tafv_status hip_error(tafv_ctx* c, hipError_t e, const char* what) { return hip_fail(c, e, what); }

void free_dev_mesh(tafv_ctx* c, DevMesh* m) { free_mesh(c, m); }

// Buffers must be at least 256-byte aligned: the kernels use 16-byte vector
// accesses and the counter slots are 128 bytes apart.
constexpr uintptr_t kAllocAlign = 256;

hipError_t dev_malloc(tafv_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  bytes = std::max<size_t>(bytes, 1);
  if (c->alloc_fn) {
    void* q = c->alloc_fn(bytes, c->alloc_user);
    if (!q) return hipErrorOutOfMemory;
    if ((uintptr_t)q % kAllocAlign) {
      c->dealloc_fn(q, c->alloc_user);
      return hipErrorInvalidValue;
    }
    *p = q;
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return e;
    }
  }
  ++c->live_buffers;
  return hipSuccess;
}

void dev_free(tafv_ctx* c, void* p) {
  if (!p) return;
  if (c->alloc_fn) c->dealloc_fn(p, c->alloc_user);
  else (void)hipFree(p);
  --c->live_buffers;
}

tafv_status read_slot_counters(tafv_ctx* c, DevMesh& m, tafv_stats* st) {
  std::vector<unsigned long long> cnt(kCounterWords);
  std::vector<double> imp(kCounterWords);
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), m.dcount, kCounterWords * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(imp.data(), m.dimpulse, kCounterWords * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream));
  std::vector<unsigned long long> nh(kCounterSlots * kNewtonWords);
  HIP_TRY(c, hipMemcpyAsync(nh.data(), m.dnewton, nh.size() * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 24; ++k) st->newton_hist[k / 8][k % 8] = 0;
  for (int k = 0; k < 3; ++k) st->newton_hist_long_updates[k] = 0;
  for (int sl = 0; sl < kCounterSlots; ++sl) {
    for (int k = 0; k < 24; ++k) st->newton_hist[k / 8][k % 8] += (int64_t)nh[sl * kNewtonWords + k];
    for (int k = 0; k < 3; ++k)
      st->newton_hist_long_updates[k] += (int64_t)nh[sl * kNewtonWords + 24 + k];
  }
  unsigned long long tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double itot[3] = {0, 0, 0};
  for (int sl = 0; sl < kCounterSlots; ++sl) {
    for (int k = 0; k < 8; ++k) tot[k] += cnt[sl * kCounterStride + k];
    for (int k = 0; k < 3; ++k) itot[k] += imp[sl * kCounterStride + k];
  }
  st->newton_updates = (int64_t)tot[0];
  st->newton_fallbacks = (int64_t)tot[1];
  st->vacuum_faces = (int64_t)tot[2];
  st->guess_faces = (int64_t)tot[3];
  st->guess_newton_updates = (int64_t)tot[4];
  st->guess_rejected = (int64_t)tot[5];
  st->guess_used = (int64_t)tot[6];
  st->guess_evaluated = (int64_t)tot[7];
  for (int k = 0; k < 3; ++k) st->wall_impulse[k] = itot[k];
  return TAFV_OK;
}

}  // namespace tafv

namespace tafv {
// device arrays of a preprocessed mesh
tafv_status upload_host_mesh(tafv_ctx* c, const HostMesh& hm, DevMesh** out) {
  *out = nullptr;
  DevMesh* m = new (std::nothrow) DevMesh();
  if (!m) return fail(c, TAFV_E_OOM, "host allocation failed");
  m->nc = (int32_t)hm.nc;
  m->nf = (int32_t)hm.nf;
  m->nb = (int32_t)hm.nbnd;
  m->ncolours = hm.ncolours;
  m->max_levels = c->prm.max_levels;
  m->scatter = c->prm.scatter;
  for (int k = 0; k <= kMaxColours; ++k) m->colour_start[k] = hm.colour_start[k];
  const size_t nc = hm.nc, nf = hm.nf;
  std::vector<float> f32;
  auto up = [&](auto* dst, const auto& src) {
    return hipMemcpy(dst, src.data(), src.size() * sizeof(src[0]), hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(dalloc(c, &m->fhL, nf));
  chk(dalloc(c, &m->fhR, nf));
  chk(dalloc(c, &m->fcol, nf));
  chk(dalloc(c, &m->fA, 3 * nf));
  chk(dalloc(c, &m->fA32, 3 * nf));
  chk(dalloc(c, &m->nb_, 4 * nc));
  chk(dalloc(c, &m->c2f, 4 * nc));
  chk(dalloc(c, &m->grc, 12 * nc));
  chk(dalloc(c, &m->grc32, 12 * nc));
  chk(dalloc(c, &m->vol, nc));
  chk(dalloc(c, &m->vol0, nc));
  chk(dalloc(c, &m->fnode, 3 * nf));
  chk(dalloc(c, &m->U, 5 * nc));
  chk(dalloc(c, &m->U0, 5 * nc));
  chk(dalloc(c, &m->R, 5 * nc));
  chk(dalloc(c, &m->lev, nc));
  chk(dalloc(c, &m->lev2, nc));
  chk(dalloc(c, &m->sweepf, kMaxLevels));
  chk(dalloc(c, &m->dt, nc));
  size_t wfbytes = (c->prm.precision == TAFV_FP32_FLUX ? sizeof(float) : sizeof(double)) * 20 * nc;
  if (c->prm.order == 2) chk(dev_malloc(c, &m->Wf, wfbytes));
  for (Partition* p : {&m->pf, &m->pc}) {  // the gather's list is scanned with the tau_g list
    int64_t n = (p == &m->pf) ? (int64_t)nf : (int64_t)nc;
    chk(dalloc(c, &p->tot, kMaxKeys));
    chk(dalloc(c, &p->offs, (size_t)kMaxKeys * partition_blocks(n)));
    chk(dalloc(c, &p->list, n));
    chk(dalloc(c, &p->counts, (size_t)kMaxKeys * partition_blocks(n)));
    chk(dalloc(c, &p->start, kMaxKeys + 1));
  }
  chk(dalloc(c, &m->pg.list, nc));
  chk(dalloc(c, &m->pg.start, kMaxKeys + 1));
  chk(dalloc(c, &m->frec, nf));
  if (m->scatter == TAFV_SCATTER_GATHER)
    chk(dev_malloc(c, &m->Q, (c->prm.precision == TAFV_FP32_FLUX ? sizeof(float) : sizeof(double)) *
                             5 * std::max<size_t>(nf, 1)));
  if (c->prm.time_order == 2) {
    chk(dev_malloc(c, &m->Q0, (c->prm.precision == TAFV_FP32_FLUX ? sizeof(float) : sizeof(double)) *
                              5 * std::max<size_t>(nf, 1)));
    chk(dalloc(c, &m->D, 5 * nc));
    chk(dalloc(c, &m->Ut, 5 * nc));
    chk(dalloc(c, &m->nkey, nc));
  }
  chk(dalloc(c, &m->fkey, nf));
  chk(dalloc(c, &m->ckey, nc));
  chk(dalloc(c, &m->lkey, nc));
  chk(dalloc(c, &m->fpack, nc));
  chk(dalloc(c, &m->perm, nc));
  chk(dalloc(c, &m->chist, (size_t)kCounterSlots * kMaxKeys));
  chk(dalloc(c, &m->dmin, kCounterWords));
  chk(dalloc(c, &m->rb, kReadbackInts));
  chk(dalloc(c, &m->xfer, 5 * nc));
  chk(dalloc(c, &m->dscal, 4));
  chk(dalloc(c, &m->dcount, kCounterWords));
  chk(dalloc(c, &m->dnewton, kCounterSlots * kNewtonWords));
  chk(dalloc(c, &m->dimpulse, kCounterWords));
  if (e != hipSuccess) {
    free_mesh(c, m);
    return hip_fail(c, e, "device allocation for the mesh");
  }
  chk(up(m->fhL, hm.fhL));
  chk(up(m->fhR, hm.fhR));
  chk(up(m->fcol, hm.fcol));
  chk(up(m->fA, hm.fA));
  f32.assign(hm.fA.begin(), hm.fA.end());
  chk(up(m->fA32, f32));
  chk(up(m->nb_, hm.nb));
  chk(up(m->c2f, hm.c2f));
  chk(up(m->grc, hm.grc));
  f32.assign(hm.grc.begin(), hm.grc.end());
  chk(up(m->grc32, f32));
  chk(up(m->vol, hm.vol));
  chk(up(m->vol0, hm.vol));
  chk(up(m->fnode, hm.fnode));
  m->n_nodes = hm.n_nodes;
  chk(up(m->perm, hm.perm));
  if (e == hipSuccess && m->scatter == TAFV_SCATTER_GATHER && c->prm.order == 2 &&
      c->prm.time_order == 1 && c->prm.fuse_faces && !c->batch) {
    // faces with both sides in one chunk of kFuseChunk cells, and boundary
    // faces, grouped by chunk (their first cell's).  The face partition
    // then keeps them apart from the faces between chunks (key tau_f + 8).
    const int64_t chunks = (hm.nc + kFuseChunk - 1) / kFuseChunk;
    std::vector<int32_t> start(chunks + 1, 0);
    std::vector<int8_t> loc(nf, 0);
    for (size_t f = 0; f < nf; ++f) {
      const int32_t hl = hm.fhL[f], hr = hm.fhR[f];
      const int32_t L = hl >> 2, Rc = hr >= 0 ? hr >> 2 : -1;
      if (Rc < 0 || Rc / kFuseChunk == L / kFuseChunk) {
        loc[f] = 1;
        start[L / kFuseChunk + 1]++;
      }
    }
    for (int64_t k = 0; k < chunks; ++k) start[k + 1] += start[k];
    std::vector<int2> lf(start[chunks]);
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (size_t f = 0; f < nf; ++f) {
      if (!loc[f]) continue;
      const int32_t hl = hm.fhL[f], hr = hm.fhR[f];
      const int32_t L = hl >> 2, Rc = hr >= 0 ? hr >> 2 : L;
      const int32_t pos = (L % kFuseChunk) | ((hl & 3) << 8) | ((Rc % kFuseChunk) << 10) |
                          ((hr >= 0 ? hr & 3 : 0) << 18) | ((hr < 0 ? 1 : 0) << 20);
      lf[fill[L / kFuseChunk]++] = make_int2((int)f, pos);
    }
    m->n_local = start[chunks];
    // compact positions of the half-faces whose neighbour lies in another
    // chunk, in cell order and by slot within a cell
    std::vector<int32_t> xb(hm.nc), fxL(nf), fxR(nf);
    int64_t nx = 0;
    for (int64_t i = 0; i < hm.nc; ++i) {
      xb[i] = (int32_t)nx;
      for (int s4 = 0; s4 < 4; ++s4) {
        const int32_t n = hm.nb[(size_t)s4 * hm.nc + i];
        nx += (n >= 0 && n / kFuseChunk != i / kFuseChunk) ? 1 : 0;
      }
    }
    // position of half-face h (cell h >> 2, slot h & 3) in the compact array
    auto xpos = [&](int32_t h) {
      const int32_t i = h >> 2;
      int32_t x = xb[i];
      for (int s4 = 0; s4 < (h & 3); ++s4) {
        const int32_t n = hm.nb[(size_t)s4 * hm.nc + i];
        x += (n >= 0 && n / kFuseChunk != i / kFuseChunk) ? 1 : 0;
      }
      return x;
    };
    for (size_t f = 0; f < nf; ++f) {
      fxL[f] = loc[f] ? hm.fhL[f] : xpos(hm.fhL[f]);
      fxR[f] = loc[f] ? hm.fhR[f] : xpos(hm.fhR[f]);
    }
    m->nx = nx;
    chk(dalloc(c, &m->flocal, nf));
    chk(dalloc(c, &m->lf_start, chunks + 1));
    chk(dalloc(c, &m->lf_face, std::max<size_t>(lf.size(), 1)));
    chk(dalloc(c, &m->xb, std::max<int64_t>(hm.nc, 1)));
    chk(dalloc(c, &m->fxL, std::max<size_t>(nf, 1)));
    chk(dalloc(c, &m->fxR, std::max<size_t>(nf, 1)));
    chk(dev_malloc(c, &m->Wx, (c->prm.precision == TAFV_FP32_FLUX ? sizeof(float)
                                                                    : sizeof(double)) *
                                  5 * (size_t)std::max<int64_t>(nx, 1)));
    chk(up(m->flocal, loc));
    chk(up(m->lf_start, start));
    if (!lf.empty()) chk(up(m->lf_face, lf));
    if (hm.nc > 0) chk(up(m->xb, xb));
    if (nf > 0) {
      chk(up(m->fxL, fxL));
      chk(up(m->fxR, fxR));
    }
  }
  if (m->scatter == TAFV_SCATTER_GATHER && c->prm.order == 2 && c->prm.time_order == 1 &&
      c->prm.pipeline_chunks > 1 && !c->batch && hm.nc > 0 && nf > 0) {
    // chunks of consecutive cells (multiples of a block of kFuseChunk cells,
    // one launch block); the faces are in
    // the order of their lower cell, and no face may reach past the next
    // chunk (a chunk's faces need the gradients of it and the next one)
    const int K = c->prm.pipeline_chunks;
    std::vector<int32_t> pc(K + 1), pf(K + 1);
    for (int k = 0; k <= K; ++k)
      pc[k] = (int32_t)std::min<int64_t>(
          hm.nc, ((hm.nc * k / K + kFuseChunk - 1) / kFuseChunk) * kFuseChunk);
    pc[K] = (int32_t)hm.nc;
    bool ok = true;
    int64_t span = 0;
    for (size_t f = 0; f < nf && ok; ++f) {
      const int32_t lo = hm.fhL[f] >> 2;
      if (f > 0 && lo < (hm.fhL[f - 1] >> 2)) ok = false;
      if (hm.fhR[f] >= 0) span = std::max<int64_t>(span, (hm.fhR[f] >> 2) - lo);
    }
    for (int k = 0; k < K && ok; ++k)
      if (pc[k + 1] - pc[k] < span || pc[k + 1] <= pc[k]) ok = false;
    if (ok) {
      size_t f = 0;
      for (int k = 0; k <= K; ++k) {
        while (f < nf && (hm.fhL[f] >> 2) < pc[k]) ++f;
        pf[k] = (int32_t)f;
      }
      pf[K] = (int32_t)nf;
      m->pipe_k = K;
      m->pipe_c = pc;
      m->pipe_f = pf;
    }
  }
  // the time-step minimum slots start at +inf (each classification sets
  // them back once it has read them)
  chk(launch_fill_u64(c->stream, m->dmin, 0x7ff0000000000000ull, kCounterWords));
  chk(hipStreamSynchronize(c->stream));
  if (e != hipSuccess) {
    free_mesh(c, m);
    return hip_fail(c, e, "mesh upload");
  }
  *out = m;
  return TAFV_OK;
}
}  // namespace tafv

extern "C" {

tafv_status tafv_params_default(tafv_params* p) {
  if (!p) return TAFV_E_ARG;
  p->gamma = 1.4;
  p->cfl = 0.5;
  p->newton_tol = 1e-12;
  p->level_margin = 1e-9;
  p->max_levels = 5;
  p->order = 2;
  p->precision = TAFV_FP64;
  p->guess = TAFV_GUESS_TR;
  p->boundary = TAFV_BC_WALL;
  p->newton_max_iter = 50;
  p->reclassify = 1;
  p->scatter = TAFV_SCATTER_GATHER;
  p->cell_order = TAFV_ORDER_CALLER;
  p->guess_stats = 0;
  p->guess_gate = 0.0;
  p->batch = 0;
  p->guess_strength = 0.0;
  p->time_order = 1;
  p->fuse_faces = 0;
  p->pipeline_chunks = 1;
  return TAFV_OK;
}

tafv_status tafv_create(int device, const tafv_params* params, void* hip_stream,
                        tafv_ctx** out) {
  if (!out) return fail(nullptr, TAFV_E_ARG, "out is NULL");
  *out = nullptr;
  if (!params) return fail(nullptr, TAFV_E_ARG, "params is NULL");
  const tafv_params& p = *params;
  if (!(p.gamma > 1.0) || !(p.cfl > 0.0) || !(p.newton_tol > 0.0) || p.max_levels < 1 ||
      p.max_levels > kMaxLevels || (p.order != 1 && p.order != 2) ||
      (p.precision != TAFV_FP64 && p.precision != TAFV_FP32_FLUX) ||
      (p.boundary != TAFV_BC_WALL && p.boundary != TAFV_BC_TRANSMIT) || p.newton_max_iter < 1 ||
      (p.scatter != TAFV_SCATTER_COLOUR && p.scatter != TAFV_SCATTER_GATHER) ||
      (p.cell_order != TAFV_ORDER_CALLER && p.cell_order != TAFV_ORDER_MORTON) ||
      !(p.level_margin >= 0.0 && p.level_margin < 0.5))
    return fail(nullptr, TAFV_E_ARG, "invalid parameters");
  if (p.guess != TAFV_GUESS_TR && p.guess != TAFV_GUESS_MLP)
    return fail(nullptr, TAFV_E_ARG, "unknown guess mode");
  if (!(p.guess_gate >= 0.0)) return fail(nullptr, TAFV_E_ARG, "negative guess gate");
  if (!(p.guess_strength >= 0.0)) return fail(nullptr, TAFV_E_ARG, "negative guess strength");
  if (p.batch != 0 && p.batch != 1) return fail(nullptr, TAFV_E_ARG, "batch must be 0 or 1");
  if (p.batch && p.scatter != TAFV_SCATTER_GATHER)
    return fail(nullptr, TAFV_E_ARG, "the batched form needs gather scatter");
  if (p.time_order != 1 && p.time_order != 2)
    return fail(nullptr, TAFV_E_ARG, "time_order must be 1 or 2");
  if (p.fuse_faces != 0 && p.fuse_faces != 1)
    return fail(nullptr, TAFV_E_ARG, "fuse_faces must be 0 or 1");
  if (p.pipeline_chunks < 0 || p.pipeline_chunks > 64)
    return fail(nullptr, TAFV_E_ARG, "pipeline_chunks must be in 0..64");
  if (p.time_order == 2 && (p.batch || p.scatter != TAFV_SCATTER_GATHER))
    return fail(nullptr, TAFV_E_ARG,
                "the predictor/corrector form needs gather scatter and no batch");
  if (p.guess == TAFV_GUESS_MLP && (p.gamma != 1.4 || p.scatter != TAFV_SCATTER_GATHER))
    return fail(nullptr, TAFV_E_ARG, "the learned guess needs gamma 1.4 and gather scatter");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(nullptr, TAFV_E_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(nullptr, TAFV_E_ARG, "device out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  e = scratch_setup(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress (no-allocation scratch)");
  tafv_ctx* c = new (std::nothrow) tafv_ctx();
  if (!c) return fail(nullptr, TAFV_E_OOM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->prm = p;
  e = hipHostMalloc((void**)&c->hpin, 4096, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "hipHostMalloc");
  }
  e = hipEventCreateWithFlags(&c->rb_event, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipHostFree(c->hpin);
    delete c;
    return hip_fail(nullptr, e, "hipEventCreateWithFlags");
  }
  for (int k = 0; k < P_N; ++k) c->prof.push_back(ProfileClass{kProfNames[k]});
  if (p.batch) {
    c->batch = new (std::nothrow) Batch();
    if (!c->batch) {
      (void)hipEventDestroy(c->rb_event);
      (void)hipHostFree(c->hpin);
      delete c;
      return fail(nullptr, TAFV_E_OOM, "host allocation failed");
    }
  }
  *out = c;
  return TAFV_OK;
}

tafv_status tafv_destroy(tafv_ctx* c) {
  if (!c) return TAFV_E_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  batch_free(c);
  for (DevMesh* m : c->meshes) free_mesh(c, m);
  for (auto& pe : c->pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->rb_event) (void)hipEventDestroy(c->rb_event);
  void* bufs[] = {c->mlp_th, c->mlp_m, c->mlp_v, c->mlp_grad, c->mlp_gpart, c->mlp_lpart,
                  c->mlp_loss, c->mlp_w, c->log_rows, c->log_count};
  for (void* b : bufs) dev_free(c, b);
  if (c->hpin) (void)hipHostFree(c->hpin);
  delete c;
  return TAFV_OK;
}

const char* tafv_last_error(const tafv_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

tafv_status tafv_set_allocator(tafv_ctx* c, void* (*alloc)(size_t, void*),
                               void (*dealloc)(void*, void*), void* user) {
  if (!c) return TAFV_E_ARG;
  if ((alloc == nullptr) != (dealloc == nullptr))
    return fail(c, TAFV_E_ARG, "give both alloc and dealloc, or neither");
  if (c->live_buffers != 0)
    return fail(c, TAFV_E_ORDER, "the allocator can only change while the context holds no "
                                 "device memory");
  c->alloc_fn = alloc;
  c->dealloc_fn = dealloc;
  c->alloc_user = alloc ? user : nullptr;
  return TAFV_OK;
}

int64_t tafv_device_buffers(const tafv_ctx* c) { return c ? c->live_buffers : -1; }

tafv_status tafv_mesh_upload(tafv_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets,
                             const int64_t* tets, int32_t* mesh_id) {
  if (!c) return TAFV_E_ARG;
  if (!xyz || !tets || !mesh_id || n_nodes < 4 || n_tets < 1)
    return fail(c, TAFV_E_ARG, "invalid mesh arguments");
  HIP_TRY(c, hipSetDevice(c->device));
  HostMesh* hm = new (std::nothrow) HostMesh();
  if (!hm) return fail(c, TAFV_E_OOM, "host allocation failed");
  tafv_status st = build_host_mesh(n_nodes, xyz, n_tets, tets,
                                   c->prm.scatter == TAFV_SCATTER_COLOUR,
                                   c->prm.cell_order == TAFV_ORDER_MORTON, hm, &c->err);
  if (st != TAFV_OK) {
    delete hm;
    return st;
  }
  if (c->prm.batch) return batch_upload(c, hm, mesh_id);  // takes hm
  DevMesh* m = nullptr;
  st = upload_host_mesh(c, *hm, &m);
  delete hm;
  if (st != TAFV_OK) return st;
  *mesh_id = (int32_t)c->meshes.size();
  c->meshes.push_back(m);
  return TAFV_OK;
}

tafv_status tafv_mesh_inspect(int64_t n_nodes, const double* xyz, int64_t n_tets,
                              const int64_t* tets, int64_t* n_faces, int64_t* n_boundary,
                              int32_t* n_colours, int32_t* face_cells, int8_t* face_colour,
                              double* face_area, int32_t* cell_neighbours,
                              double* recon_coef) {
  if (!xyz || !tets || n_nodes < 4 || n_tets < 1) return fail(nullptr, TAFV_E_ARG, "invalid mesh");
  HostMesh hm;
  std::string err;
  tafv_status st = build_host_mesh(n_nodes, xyz, n_tets, tets, true, false, &hm, &err);
  if (st != TAFV_OK) return fail(nullptr, st, err);
  if (n_faces) *n_faces = hm.nf;
  if (n_boundary) *n_boundary = hm.nbnd;
  if (n_colours) *n_colours = hm.ncolours;
  const std::vector<int32_t>& perm = hm.perm;  // internal -> caller
  for (int64_t f = 0; f < hm.nf; ++f) {
    if (face_cells) {
      face_cells[2 * f] = perm[hm.fhL[f] >> 2];
      face_cells[2 * f + 1] = hm.fhR[f] >= 0 ? perm[hm.fhR[f] >> 2] : -1;
    }
    if (face_colour) face_colour[f] = hm.fcol[f];
    if (face_area)
      for (int k = 0; k < 3; ++k) face_area[3 * f + k] = hm.fA[k * hm.nf + f];
  }
  if (cell_neighbours)
    for (int64_t i = 0; i < hm.nc; ++i)
      for (int m = 0; m < 4; ++m) {
        int32_t n = hm.nb[m * hm.nc + i];
        cell_neighbours[4 * (int64_t)perm[i] + m] = n >= 0 ? perm[n] : -1;
      }
  if (recon_coef)
    for (int64_t i = 0; i < hm.nc; ++i)
      for (int k = 0; k < 12; ++k) recon_coef[12 * (int64_t)perm[i] + k] = hm.grc[k * hm.nc + i];
  return TAFV_OK;
}

tafv_status tafv_mesh_params(tafv_ctx* c, int32_t mesh_id, int32_t max_levels) {
  if (c && c->batch) return batch_mesh_params(c, mesh_id, max_levels);
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (max_levels < 1 || max_levels > kMaxLevels) return fail(c, TAFV_E_ARG, "max_levels out of range");
  m->max_levels = max_levels;
  m->classified = false;
  return TAFV_OK;
}

tafv_status tafv_state_init(tafv_ctx* c, int32_t mesh_id, const double* prim) {
  if (c && c->batch) return batch_state_init(c, mesh_id, prim);
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!prim) return fail(c, TAFV_E_ARG, "prim is NULL");
  for (int64_t i = 0; i < m->nc; ++i) {
    const double* w = prim + 5 * i;
    for (int k = 0; k < 5; ++k)
      if (!std::isfinite(w[k]))
        return fail(c, TAFV_E_STATE, "non-finite initial value at cell " + std::to_string(i));
    if (!(w[0] > 0.0) || !(w[4] > 0.0))
      return fail(c, TAFV_E_STATE, "rho <= 0 or p <= 0 at cell " + std::to_string(i));
  }
  HIP_TRY(c, hipSetDevice(c->device));
  hipError_t e = hipMemcpyAsync(m->xfer, prim, sizeof(double) * 5 * m->nc, hipMemcpyHostToDevice,
                                c->stream);
  if (e == hipSuccess) e = launch_state_init(c->stream, *m, m->xfer, c->prm.gamma);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->U0, m->U, sizeof(double) * 5 * m->nc, hipMemcpyDeviceToDevice,
                       c->stream);
  if (e == hipSuccess) e = sync_time_states(c, *m);
  if (e == hipSuccess) e = reset_volumes(c, *m);
  if (e == hipSuccess) e = launch_fill_u64(c->stream, m->dcount, 0ull, kCounterWords);
  if (e == hipSuccess)
    e = launch_fill_u64(c->stream, m->dnewton, 0ull, kCounterSlots * kNewtonWords);
  if (e == hipSuccess) e = launch_fill_f64(c->stream, m->dimpulse, 0.0, kCounterWords);
  if (e == hipSuccess) e = launch_fill_u64(c->stream, m->dscal, 0ull, 4);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "state init");
  m->has_state = true;
  m->phase = 0;
  m->theta = 0;
  m->t = 0.0;
  m->dt_min = 0.0;
  m->classified = false;
  m->st = tafv_stats{};
  return TAFV_OK;
}

tafv_status tafv_state_reset(tafv_ctx* c, int32_t mesh_id) {
  if (c && c->batch) return batch_state_reset(c, mesh_id);
  if (c && mesh_id == -1) {
    for (int32_t k = 0; k < (int32_t)c->meshes.size(); ++k) {
      tafv_status st = tafv_state_reset(c, k);
      if (st != TAFV_OK) return st;
    }
    return TAFV_OK;
  }
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!m->has_state) return fail(c, TAFV_E_ORDER, "no state");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(m->U, m->U0, sizeof(double) * 5 * m->nc, hipMemcpyDeviceToDevice,
                            c->stream));
  HIP_TRY(c, launch_fill_f64(c->stream, m->R, 0.0, (int64_t)5 * m->nc));
  HIP_TRY(c, sync_time_states(c, *m));
  HIP_TRY(c, reset_volumes(c, *m));
  m->phase = 0;
  m->theta = 0;
  m->t = 0.0;
  m->dt_min = 0.0;
  m->classified = false;
  return TAFV_OK;
}

}  // extern "C"

namespace {

tafv_status call_stats(tafv_ctx* c, tafv_stats acc, tafv_stats* out);

// a single-mesh-path context that can advance
tafv_status advance_ready(tafv_ctx* c) {
  if (c->batch) return fail(c, TAFV_E_ARG, "a batched context advances on its own");
  if (c->meshes.empty()) return fail(c, TAFV_E_ORDER, "no mesh uploaded");
  for (DevMesh* m : c->meshes)
    if (!m->has_state) return fail(c, TAFV_E_ORDER, "advance before state_init");
  if (c->prm.guess == TAFV_GUESS_MLP && !c->mlp_ready)
    return fail(c, TAFV_E_MLP, "learned guess selected but no network set");
  return TAFV_OK;
}

}  // namespace

extern "C" {

tafv_status tafv_advance(tafv_ctx* c, int64_t n, tafv_stats* out) {
  if (!c) return TAFV_E_ARG;
  if (n < 0) return fail(c, TAFV_E_ARG, "negative subiteration count");
  if (c->batch) return batch_advance(c, n, out);
  tafv_status rdy = advance_ready(c);
  if (rdy != TAFV_OK) return rdy;
  HIP_TRY(c, hipSetDevice(c->device));
  tafv_stats acc{};
  for (int64_t k = 0; k < n; ++k) {
    for (DevMesh* m : c->meshes) {
      tafv_status st = subiteration(c, *m, &acc);
      if (st != TAFV_OK) return st;
    }
  }
  return out ? call_stats(c, acc, out) : TAFV_OK;
}

tafv_status tafv_advance_group(tafv_ctx* const* ctxs, int32_t n, int64_t n_dt_min,
                               int32_t workers, tafv_stats* out) {
  if (!ctxs || n < 1 || n_dt_min < 0 || workers < 1)
    return fail(nullptr, TAFV_E_ARG, "invalid group arguments");
  std::set<const tafv_ctx*> seen;
  for (int32_t i = 0; i < n; ++i) {
    tafv_ctx* c = ctxs[i];
    if (!c || !seen.insert(c).second)
      return fail(nullptr, TAFV_E_ARG, "a group needs distinct non-NULL contexts");
    tafv_status st = advance_ready(c);
    if (st != TAFV_OK) return st;
  }
  workers = std::min(workers, n);
  std::atomic<bool> stop{false};
  std::vector<tafv_status> res(n, TAFV_OK);
  std::vector<tafv_stats> acc(n, tafv_stats{});
  // worker w drives contexts w, w + workers, ...: one subiteration of each
  // in turn, so every context's stream keeps queued work while one of them
  // waits for its iteration-start readback, and no context waits for the
  // others at a subiteration boundary
  auto work = [&](int w) {
    for (int64_t k = 0; k < n_dt_min && !stop.load(std::memory_order_relaxed); ++k)
      for (int32_t i = w; i < n; i += workers) {
        tafv_ctx* c = ctxs[i];
        hipError_t e = hipSetDevice(c->device);
        tafv_status st = e == hipSuccess ? TAFV_OK : hip_fail(c, e, "hipSetDevice");
        for (DevMesh* m : c->meshes)
          if (st == TAFV_OK) st = subiteration(c, *m, &acc[i]);
        if (st != TAFV_OK) {
          res[i] = st;
          stop.store(true);
          return;
        }
      }
  };
  std::vector<std::thread> pool;
  try {
    for (int w = 1; w < workers; ++w) pool.emplace_back(work, w);
  } catch (...) {  // fewer threads: the ones started and this one share the work
    stop.store(true);
  }
  if (!stop.load()) work(0);
  for (std::thread& t : pool) t.join();
  if (pool.size() + 1 < (size_t)workers && std::all_of(res.begin(), res.end(), [](tafv_status x) {
        return x == TAFV_OK;
      }))
    return fail(nullptr, TAFV_E_ARG, "could not start the worker threads");
  for (int32_t i = 0; i < n; ++i)
    if (res[i] != TAFV_OK) return res[i];
  if (!out) return TAFV_OK;
  tafv_stats tot{};
  for (int32_t i = 0; i < n; ++i) {
    tafv_stats one{};
    tafv_status st = call_stats(ctxs[i], acc[i], &one);
    if (st != TAFV_OK) return st;
    tot.subiterations += one.subiterations;
    tot.cell_updates += one.cell_updates;
    tot.face_solves += one.face_solves;
    tot.newton_updates += one.newton_updates;
    tot.newton_fallbacks += one.newton_fallbacks;
    tot.vacuum_faces += one.vacuum_faces;
    tot.guess_faces += one.guess_faces;
    tot.guess_newton_updates += one.guess_newton_updates;
    tot.guess_rejected += one.guess_rejected;
    tot.guess_used += one.guess_used;
    tot.guess_evaluated += one.guess_evaluated;
    for (int k = 0; k < 3; ++k) tot.wall_impulse[k] += one.wall_impulse[k];
    for (int k = 0; k < 24; ++k) tot.newton_hist[k / 8][k % 8] += one.newton_hist[k / 8][k % 8];
    for (int k = 0; k < 3; ++k) tot.newton_hist_long_updates[k] += one.newton_hist_long_updates[k];
    for (int t = 0; t < kMaxLevels; ++t) tot.cells_per_level[t] += one.cells_per_level[t];
    tot.theta = std::max(tot.theta, one.theta);
    tot.phase = one.phase;
    tot.dt_min = one.dt_min;
    tot.t_reached = one.t_reached;
  }
  *out = tot;
  return TAFV_OK;
}

}  // extern "C"

namespace {

// The counters of one tafv_advance call (acc) completed with the device
// counters of the context's meshes and the schedule state of its last mesh.
tafv_status call_stats(tafv_ctx* c, tafv_stats acc, tafv_stats* out) {
  for (DevMesh* m : c->meshes) {
    tafv_status st = read_counters(c, *m);
    if (st != TAFV_OK) return st;
  }
  {
    DevMesh* last = c->meshes.back();
    acc.theta = last->theta;
    acc.phase = last->phase;
    acc.dt_min = last->dt_min;
    acc.t_reached = last->t;
    for (int t = 0; t < kMaxLevels; ++t) acc.cells_per_level[t] = last->st.cells_per_level[t];
    for (DevMesh* m : c->meshes) {
      acc.newton_updates += m->st.newton_updates;
      acc.newton_fallbacks += m->st.newton_fallbacks;
      acc.vacuum_faces += m->st.vacuum_faces;
      acc.guess_faces += m->st.guess_faces;
      acc.guess_newton_updates += m->st.guess_newton_updates;
      acc.guess_rejected += m->st.guess_rejected;
      acc.guess_used += m->st.guess_used;
      acc.guess_evaluated += m->st.guess_evaluated;
      for (int k = 0; k < 3; ++k) acc.wall_impulse[k] += m->st.wall_impulse[k];
      for (int k = 0; k < 24; ++k) acc.newton_hist[k / 8][k % 8] += m->st.newton_hist[k / 8][k % 8];
      for (int k = 0; k < 3; ++k)
        acc.newton_hist_long_updates[k] += m->st.newton_hist_long_updates[k];
    }
    *out = acc;
  }
  return TAFV_OK;
}

}  // namespace

extern "C" {

tafv_status tafv_mesh_stats(tafv_ctx* c, int32_t mesh_id, tafv_stats* out) {
  if (c && c->batch) return batch_mesh_stats(c, mesh_id, out);
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!out) return fail(c, TAFV_E_ARG, "out is NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  tafv_status st = read_counters(c, *m);
  if (st != TAFV_OK) return st;
  *out = m->st;
  return TAFV_OK;
}

tafv_status tafv_state_read(tafv_ctx* c, int32_t mesh_id, double* cons, int8_t* levels) {
  if (c && c->batch) return batch_state_read(c, mesh_id, cons, levels);
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!cons) return fail(c, TAFV_E_ARG, "cons is NULL");
  if (!m->has_state) return fail(c, TAFV_E_ORDER, "no state");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_to_caller_f64(c->stream, *m, m->U, m->xfer));
  HIP_TRY(c, hipMemcpyAsync(cons, m->xfer, sizeof(double) * 5 * m->nc, hipMemcpyDeviceToHost,
                            c->stream));
  if (levels) {
    int8_t* stage = (int8_t*)m->xfer;
    HIP_TRY(c, launch_to_caller_i8(c->stream, *m, m->lev, stage));
    HIP_TRY(c, hipMemcpyAsync(levels, stage, m->nc, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

tafv_status tafv_checkpoint_read(tafv_ctx* c, int32_t mesh_id, double* cons, double* accum,
                                 int8_t* levels, int32_t* phase, int32_t* theta, double* dt_min,
                                 double* t) {
  if (c && c->batch)
    return batch_checkpoint_read(c, mesh_id, cons, accum, levels, phase, theta, dt_min, t);
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!cons || !accum || !levels || !phase || !theta || !dt_min || !t)
    return fail(c, TAFV_E_ARG, "NULL argument");
  if (!m->has_state) return fail(c, TAFV_E_ORDER, "no state");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_to_caller_f64(c->stream, *m, m->U, m->xfer));
  HIP_TRY(c, hipMemcpyAsync(cons, m->xfer, sizeof(double) * 5 * m->nc, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, launch_to_caller_f64(c->stream, *m, m->R, m->xfer));
  HIP_TRY(c, hipMemcpyAsync(accum, m->xfer, sizeof(double) * 5 * m->nc, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, launch_to_caller_i8(c->stream, *m, m->lev, (int8_t*)m->xfer));
  HIP_TRY(c, hipMemcpyAsync(levels, m->xfer, m->nc, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *phase = m->phase;
  *theta = m->theta;
  *dt_min = m->dt_min;
  *t = m->t;
  return TAFV_OK;
}

tafv_status tafv_checkpoint_write(tafv_ctx* c, int32_t mesh_id, const double* cons,
                                  const double* accum, const int8_t* levels, int32_t phase,
                                  int32_t theta, double dt_min, double t) {
  if (c && c->batch) return fail(c, TAFV_E_ARG, "checkpoints are not available in the batched form");
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return c ? fail(c, TAFV_E_ARG, "unknown mesh") : TAFV_E_ARG;
  if (!cons || !accum || !levels) return fail(c, TAFV_E_ARG, "NULL argument");
  if (theta < 0 || theta >= m->max_levels || phase < 0 || phase >= (1 << theta) ||
      !(dt_min > 0.0))
    return fail(c, TAFV_E_ARG, "invalid schedule state");
  if (c->prm.time_order == 2 && phase != 0)
    return fail(c, TAFV_E_ARG,
                "predictor/corrector form: checkpoints are written at phase 0 only");
  if (m->moving)
    return fail(c, TAFV_E_ARG, "checkpoints are not written on moving meshes");
  for (int64_t i = 0; i < m->nc; ++i)
    if (levels[i] < 0 || levels[i] > theta) return fail(c, TAFV_E_ARG, "level out of range");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(m->xfer, cons, sizeof(double) * 5 * m->nc, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, launch_from_caller_f64(c->stream, *m, m->xfer, m->U));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpyAsync(m->xfer, accum, sizeof(double) * 5 * m->nc, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, launch_from_caller_f64(c->stream, *m, m->xfer, m->R));
  HIP_TRY(c, sync_time_states(c, *m));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpyAsync(m->xfer, levels, m->nc, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_from_caller_i8(c->stream, *m, (const int8_t*)m->xfer, m->lev));
  // the level histogram starts from zero; the kernels read dt_min on the device
  HIP_TRY(c, launch_fill_u64(c->stream, (unsigned long long*)m->chist, 0ull,
                             kCounterSlots * kMaxKeys / 2));
  unsigned long long dbits;
  std::memcpy(&dbits, &dt_min, sizeof(dbits));
  HIP_TRY(c, launch_fill_u64(c->stream, m->dscal, dbits, 1));
  m->split_local = fusable(c, *m, flux_features(c, *m));
  HIP_TRY(c, launch_partitions(c->stream, *m, early_order(c, *m)));
  int K = face_list_keys(*m);
  HIP_TRY(c, hipMemcpyAsync(m->hstart_f, m->pf.start, (K + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(m->hstart_c, m->pc.start, (kMaxLevels + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(m->hstart_g, m->pg.start, (kCellKeys + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->hpin, m->rb, kReadbackInts * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(m->hhist, c->hpin + kRbHist, kMaxKeys * sizeof(int32_t));
  level_histogram(*m);
  m->has_state = true;
  m->phase = phase;
  m->theta = theta;
  m->dt_min = dt_min;
  m->t = t;
  m->classified = true;
  return TAFV_OK;
}

tafv_status tafv_guess_config(tafv_ctx* c, int32_t guess, double gate, double strength,
                              int32_t stats) {
  if (!c) return TAFV_E_ARG;
  if (guess != TAFV_GUESS_TR && guess != TAFV_GUESS_MLP) return fail(c, TAFV_E_ARG, "unknown guess");
  if (!(gate >= 0.0)) return fail(c, TAFV_E_ARG, "negative guess gate");
  if (!(strength >= 0.0)) return fail(c, TAFV_E_ARG, "negative guess strength");
  if (guess == TAFV_GUESS_MLP && (c->prm.gamma != 1.4 || c->prm.scatter != TAFV_SCATTER_GATHER))
    return fail(c, TAFV_E_ARG, "the learned guess needs gamma 1.4 and gather scatter");
  if ((guess != TAFV_GUESS_TR || stats) && any_moving(c))
    return fail(c, TAFV_E_ARG, "moving meshes take the two-rarefaction start without statistics");
  c->prm.guess = guess;
  c->prm.guess_gate = gate;
  c->prm.guess_strength = strength;
  c->prm.guess_stats = stats != 0;
  if (c->batch) batch_invalidate(c);
  return TAFV_OK;
}

tafv_status tafv_mesh_motion(tafv_ctx* c, int32_t mesh_id, const double* node_vel) {
  if (!c) return TAFV_E_ARG;
  if (c->batch) return fail(c, TAFV_E_ARG, "moving meshes are not available in the batched form");
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return fail(c, TAFV_E_ARG, "unknown mesh");
  if (!node_vel) return fail(c, TAFV_E_ARG, "node_vel is NULL");
  if (c->prm.time_order != 1 || m->scatter != TAFV_SCATTER_GATHER)
    return fail(c, TAFV_E_ARG, "moving meshes need time_order 1 and gather scatter");
  if (c->prm.guess != TAFV_GUESS_TR || c->prm.guess_stats || c->log_cap > 0)
    return fail(c, TAFV_E_ARG,
                "moving meshes take the two-rarefaction start, without statistics or logging");
  for (int64_t k = 0; k < 3 * m->n_nodes; ++k)
    if (!std::isfinite(node_vel[k])) return fail(c, TAFV_E_ARG, "non-finite node velocity");
  HIP_TRY(c, hipSetDevice(c->device));
  if (!m->sF) {
    HIP_TRY(c, dalloc(c, &m->sF, std::max<int64_t>(m->nf, 1)));
    HIP_TRY(c, dalloc(c, &m->Rv, std::max<int64_t>(m->nc, 1)));
    HIP_TRY(c, launch_fill_f64(c->stream, m->Rv, 0.0, m->nc));
  }
  double* dvel = nullptr;
  const size_t bytes = sizeof(double) * 3 * (size_t)std::max<int64_t>(m->n_nodes, 1);
  HIP_TRY(c, dev_alloc(c, &dvel, bytes));
  hipError_t e = hipMemcpyAsync(dvel, node_vel, sizeof(double) * 3 * m->n_nodes,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_face_speed(c->stream, *m, dvel);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, dvel);
  if (e != hipSuccess) return hip_fail(c, e, "mesh motion");
  m->moving = true;
  return TAFV_OK;
}

tafv_status tafv_volume_read(tafv_ctx* c, int32_t mesh_id, double* vol) {
  if (!c) return TAFV_E_ARG;
  if (c->batch) return fail(c, TAFV_E_ARG, "moving meshes are not available in the batched form");
  DevMesh* m = get_mesh(c, mesh_id);
  if (!m) return fail(c, TAFV_E_ARG, "unknown mesh");
  if (!vol) return fail(c, TAFV_E_ARG, "vol is NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_vol_to_caller(c->stream, *m, m->vol, m->xfer));
  HIP_TRY(c, hipMemcpyAsync(vol, m->xfer, sizeof(double) * m->nc, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

static tafv_status ensure_mlp(tafv_ctx* c) {
  if (c->mlp_th) return TAFV_OK;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(dev_alloc(c, &c->mlp_th, kMlpParams * sizeof(float)));
  chk(dev_alloc(c, &c->mlp_m, kMlpParams * sizeof(float)));
  chk(dev_alloc(c, &c->mlp_v, kMlpParams * sizeof(float)));
  chk(dev_alloc(c, &c->mlp_grad, kMlpParams * sizeof(float)));
  chk(dev_alloc(c, &c->mlp_loss, 4096 * sizeof(float)));
  chk(dev_alloc(c, &c->mlp_w, sizeof(MlpDev)));
  if (e != hipSuccess) {  // all or nothing: the next call starts over
    for (float** q : {&c->mlp_th, &c->mlp_m, &c->mlp_v, &c->mlp_grad, &c->mlp_loss}) {
      dev_free(c, *q);
      *q = nullptr;
    }
    dev_free(c, c->mlp_w);
    c->mlp_w = nullptr;
    return hip_fail(c, e, "network allocation");
  }
  return TAFV_OK;
}

static tafv_status ensure_gpart(tafv_ctx* c, int64_t rows) {
  int64_t nb = (rows + 63) / 64;
  if (nb <= c->mlp_gpart_blocks) return TAFV_OK;
  dev_free(c, c->mlp_gpart);
  dev_free(c, c->mlp_lpart);
  c->mlp_gpart = nullptr;
  c->mlp_lpart = nullptr;
  c->mlp_gpart_blocks = 0;
  HIP_TRY(c, dev_alloc(c, &c->mlp_gpart, (size_t)nb * kMlpParams * sizeof(float)));
  HIP_TRY(c, dev_alloc(c, &c->mlp_lpart, (size_t)nb * sizeof(float)));
  c->mlp_gpart_blocks = nb;
  return TAFV_OK;
}

// device copies of host rows for the network calls, freed on scope exit
struct DevBuf {
  tafv_ctx* c;
  void* p = nullptr;
  explicit DevBuf(tafv_ctx* c_) : c(c_) {}
  ~DevBuf() { dev_free(c, p); }
};

tafv_status tafv_mlp_set(tafv_ctx* c, const float* params, int64_t n) {
  if (!c) return TAFV_E_ARG;
  if (!params || n != kMlpParams) return fail(c, TAFV_E_ARG, "expected 1313 parameters");
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(params[k])) return fail(c, TAFV_E_MLP, "non-finite network parameter");
  HIP_TRY(c, hipSetDevice(c->device));
  tafv_status st = ensure_mlp(c);
  if (st != TAFV_OK) return st;
  HIP_TRY(c, hipMemcpyAsync(c->mlp_th, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, mlp_fill(c->stream, c->mlp_m, 0.f, kMlpParams));
  HIP_TRY(c, mlp_fill(c->stream, c->mlp_v, 0.f, kMlpParams));
  HIP_TRY(c, mlp_pack(c->stream, c->mlp_th, (MlpDev*)c->mlp_w));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_step = 0;
  c->mlp_ready = true;
  return TAFV_OK;
}

tafv_status tafv_mlp_get(tafv_ctx* c, float* params, int64_t n) {
  if (!c) return TAFV_E_ARG;
  if (!params || n != kMlpParams) return fail(c, TAFV_E_ARG, "expected 1313 parameters");
  if (!c->mlp_ready) return fail(c, TAFV_E_MLP, "no network set");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(params, c->mlp_th, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

tafv_status tafv_mlp_forward(tafv_ctx* c, const float* x, int64_t n, float* y) {
  if (!c) return TAFV_E_ARG;
  if (!x || !y || n < 0 || n > INT32_MAX / 8) return fail(c, TAFV_E_ARG, "invalid arguments");
  if (!c->mlp_ready) return fail(c, TAFV_E_MLP, "no network set");
  if (n == 0) return TAFV_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  DevBuf dx(c), dy(c);
  HIP_TRY(c, dev_malloc(c, &dx.p, n * kMlpIn * sizeof(float)));
  HIP_TRY(c, dev_malloc(c, &dy.p, n * sizeof(float)));
  HIP_TRY(c, hipMemcpyAsync(dx.p, x, n * kMlpIn * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mlp_forward(c->stream, (int)n, (const float*)dx.p, (const MlpDev*)c->mlp_w,
                         (float*)dy.p));
  HIP_TRY(c, hipMemcpyAsync(y, dy.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

tafv_status tafv_mlp_grad(tafv_ctx* c, const float* x, const float* t, int64_t n, float* grad,
                          float* loss) {
  if (!c) return TAFV_E_ARG;
  if (!x || !t || n < 1 || n > INT32_MAX / 8) return fail(c, TAFV_E_ARG, "invalid arguments");
  if (!c->mlp_ready) return fail(c, TAFV_E_MLP, "no network set");
  HIP_TRY(c, hipSetDevice(c->device));
  tafv_status st = ensure_gpart(c, n);
  if (st != TAFV_OK) return st;
  DevBuf dx(c), dt(c);
  HIP_TRY(c, dev_malloc(c, &dx.p, n * kMlpIn * sizeof(float)));
  HIP_TRY(c, dev_malloc(c, &dt.p, n * sizeof(float)));
  HIP_TRY(c, hipMemcpyAsync(dx.p, x, n * kMlpIn * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(dt.p, t, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mlp_fill(c->stream, c->mlp_loss, 0.f, 1));
  HIP_TRY(c, mlp_gradient(c->stream, 1ull, 0ull, (unsigned long long)n, 0, n, (const float*)dx.p,
                          (const float*)dt.p, (const MlpDev*)c->mlp_w, c->mlp_gpart,
                          c->mlp_lpart, c->mlp_grad, c->mlp_loss, 1.0f / (float)n));
  if (grad)
    HIP_TRY(c, hipMemcpyAsync(grad, c->mlp_grad, kMlpParams * sizeof(float),
                              hipMemcpyDeviceToHost, c->stream));
  float l = 0.f;
  HIP_TRY(c, hipMemcpyAsync(&l, c->mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return TAFV_OK;
}

tafv_status tafv_mlp_grad_noalloc(tafv_ctx* c, const float* x, const float* t, int64_t n,
                                  float* grad, float* loss) {
  if (!c) return TAFV_E_ARG;
  if (!x || !t || n < 1) return fail(c, TAFV_E_ARG, "invalid arguments");
  if (n > kScrRows)
    return fail(c, TAFV_E_ARG, "more rows than the no-allocation scratch holds");
  if (!c->mlp_ready) return fail(c, TAFV_E_MLP, "no network set");
  HIP_TRY(c, hipSetDevice(c->device));
  float* base = scratch_ptr(c->device);
  if (!base) return fail(c, TAFV_E_DEVICE, "no-allocation scratch not set up on this device");
  float *sx = base + kScrX, *st = base + kScrT, *sgrad = base + kScrGrad, *sloss = base + kScrLoss;
  HIP_TRY(c, hipMemcpyAsync(sx, x, n * kMlpIn * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(st, t, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mlp_fill(c->stream, sloss, 0.f, 1));
  HIP_TRY(c, mlp_gradient(c->stream, 1ull, 0ull, (unsigned long long)n, 0, n, sx, st,
                          (const MlpDev*)c->mlp_w, base + kScrGpart, base + kScrLpart, sgrad,
                          sloss, 1.0f / (float)n));
  if (grad)
    HIP_TRY(c, hipMemcpyAsync(grad, sgrad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
  float l = 0.f;
  HIP_TRY(c, hipMemcpyAsync(&l, sloss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return TAFV_OK;
}

static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

tafv_status tafv_mlp_train(tafv_ctx* c, const float* x, const float* t, int64_t n,
                           int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss) {
  if (!c) return TAFV_E_ARG;
  if (!x || !t || n < 1 || n > INT32_MAX / 8 || epochs < 0 || epochs > 4096 || batch < 1 ||
      !(lr > 0.f))
    return fail(c, TAFV_E_ARG, "invalid arguments");
  if (!c->mlp_ready) return fail(c, TAFV_E_MLP, "no network set (initial parameters)");
  HIP_TRY(c, hipSetDevice(c->device));
  tafv_status st = ensure_gpart(c, std::min<int64_t>(batch, n));
  if (st != TAFV_OK) return st;
  DevBuf dx(c), dt(c);
  HIP_TRY(c, dev_malloc(c, &dx.p, n * kMlpIn * sizeof(float)));
  HIP_TRY(c, dev_malloc(c, &dt.p, n * sizeof(float)));
  HIP_TRY(c, hipMemcpyAsync(dx.p, x, n * kMlpIn * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(dt.p, t, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mlp_fill(c->stream, c->mlp_loss, 0.f, std::max(epochs, 1)));
  uint64_t state = seed;
  for (int e = 0; e < epochs; ++e) {
    uint64_t un = (uint64_t)n;
    uint64_t a = un > 2 ? 1 + 2 * (splitmix64(state) % (un / 2)) : 1;
    while (gcd_u64(a, un) != 1) a += 2;
    uint64_t b = splitmix64(state) % un;
    for (int64_t first = 0; first < n; first += batch) {
      int64_t cnt = std::min<int64_t>(batch, n - first);
      HIP_TRY(c, mlp_gradient(c->stream, a, b, un, first, cnt, (const float*)dx.p,
                              (const float*)dt.p, (const MlpDev*)c->mlp_w, c->mlp_gpart,
                              c->mlp_lpart, c->mlp_grad, c->mlp_loss + e, 1.0f / (float)n));
      HIP_TRY(c, mlp_adam(c->stream, c->mlp_th, c->mlp_m, c->mlp_v, c->mlp_grad, lr,
                          ++c->mlp_step));
      HIP_TRY(c, mlp_pack(c->stream, c->mlp_th, (MlpDev*)c->mlp_w));
    }
  }
  if (loss && epochs > 0)
    HIP_TRY(c, hipMemcpyAsync(loss, c->mlp_loss, epochs * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TAFV_OK;
}

tafv_status tafv_facelog_config(tafv_ctx* c, int64_t capacity, double rate, uint64_t seed) {
  if (!c) return TAFV_E_ARG;
  if (capacity < 0 || !(rate >= 0.0 && rate <= 1.0)) return fail(c, TAFV_E_ARG, "invalid log");
  if (c->batch && capacity > 0)
    return fail(c, TAFV_E_ARG, "face logging is not available in the batched form");
  if (capacity > 0 && any_moving(c))
    return fail(c, TAFV_E_ARG, "face logging is not available on moving meshes");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, c->log_rows);
  c->log_rows = nullptr;
  c->log_cap = 0;
  if (!c->log_count) HIP_TRY(c, dev_alloc(c, &c->log_count, sizeof(unsigned long long)));
  HIP_TRY(c, launch_fill_u64(c->stream, c->log_count, 0ull, 1));
  if (capacity > 0) HIP_TRY(c, dev_alloc(c, &c->log_rows, (size_t)capacity * 7 * sizeof(float)));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->log_cap = capacity;
  c->log_rate = rate;
  c->log_seed = seed;
  return TAFV_OK;
}

tafv_status tafv_facelog_read(tafv_ctx* c, float* rows, int64_t cap, int64_t* n_rows) {
  if (!c) return TAFV_E_ARG;
  if (!n_rows || cap < 0 || (cap > 0 && !rows)) return fail(c, TAFV_E_ARG, "invalid arguments");
  *n_rows = 0;
  if (!c->log_count) return TAFV_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  unsigned long long cnt = 0;
  HIP_TRY(c, hipMemcpyAsync(&cnt, c->log_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // The waves take row slots in the order they reach the counter, which
  // varies from run to run; the rows held are returned sorted by their
  // bytes, so that a run's rows (and what is trained on them) do not
  // depend on it.
  const int64_t held = (int64_t)std::min<unsigned long long>(cnt, (unsigned long long)c->log_cap);
  const int64_t k = std::min<int64_t>(held, cap);
  if (k > 0) {
    std::vector<float> all((size_t)held * 7);
    HIP_TRY(c, hipMemcpyAsync(all.data(), c->log_rows, all.size() * sizeof(float),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<int64_t> order((size_t)held);
    for (int64_t r = 0; r < held; ++r) order[(size_t)r] = r;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return std::memcmp(&all[(size_t)a * 7], &all[(size_t)b * 7], 7 * sizeof(float)) < 0;
    });
    for (int64_t r = 0; r < k; ++r)
      std::memcpy(rows + (size_t)r * 7, &all[(size_t)order[(size_t)r] * 7], 7 * sizeof(float));
  }
  *n_rows = k;
  return TAFV_OK;
}

tafv_status tafv_profile_enable(tafv_ctx* c, int32_t on) {
  if (!c) return TAFV_E_ARG;
  c->profile = on != 0;
  return TAFV_OK;
}

tafv_status tafv_profile_read(tafv_ctx* c, int32_t n, double* ms, int64_t* launches,
                              int64_t* items, const char** names, int32_t* n_classes) {
  if (!c) return TAFV_E_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto& pe : c->pending) {
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, pe.a, pe.b));
    c->prof[pe.cls].ms += t;
    c->prof[pe.cls].launches += 1;
    c->prof[pe.cls].items += pe.items;
    c->event_pool.push_back(pe.a);
    c->event_pool.push_back(pe.b);
  }
  c->pending.clear();
  int nc = (int)c->prof.size();
  if (n_classes) *n_classes = nc;
  for (int k = 0; k < std::min(n, nc); ++k) {
    if (ms) ms[k] = c->prof[k].ms;
    if (launches) launches[k] = c->prof[k].launches;
    if (items) items[k] = c->prof[k].items;
    if (names) names[k] = c->prof[k].name;
    c->prof[k].ms = 0.0;
    c->prof[k].launches = 0;
    c->prof[k].items = 0;
  }
  return TAFV_OK;
}

tafv_status tafv_batch_config(tafv_ctx* c, int32_t graph, int32_t autotune,
                              const char* tune_cache) {
  if (!c) return TAFV_E_ARG;
  if (!c->batch) return fail(c, TAFV_E_ARG, "not a batched context");
  return batch_config(c, graph, autotune, tune_cache);
}

tafv_status tafv_batch_info(tafv_ctx* c, int32_t* info, int32_t n) {
  if (!c) return TAFV_E_ARG;
  if (!c->batch) return fail(c, TAFV_E_ARG, "not a batched context");
  return batch_info(c, info, n);
}

}  // extern "C"
