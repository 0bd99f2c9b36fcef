// Launchers of the device kernels (defined in kernels.hip).
#pragma once

#include "gas.h"
#include "mlp.h"
#include "tafv_internal.h"

namespace tafv {

// The cells a launch takes from a cell list: the first n1 entries, then n2
// entries from off2 on (see list_cell).
struct CellRange {
  int n1 = 0, off2 = 0, n2 = 0;
  int count() const { return n1 + n2; }
};

// Up to kMaxLevels + 1 ranges of a cell list: range r holds items
// cum[r] .. cum[r + 1] - 1, at list[off[r] + item - cum[r]] (see range_cell).
struct ListRanges {
  int n = 0;
  int off[kMaxLevels + 1] = {0};
  int cum[kMaxLevels + 2] = {0};
  void add(int a, int b) {  // entries [a, b) of the list
    if (b <= a) return;
    if (n > 0 && off[n - 1] + (cum[n] - cum[n - 1]) == a) {
      cum[n] += b - a;  // continues the previous range
      return;
    }
    off[n] = a;
    cum[n + 1] = cum[n] + (b - a);
    ++n;
  }
  int count() const { return cum[n]; }
};

// Per-launch parameters shared by the face and cell kernels.
struct StepArgs {
  Gas gas;
  double cfl, newton_tol, level_margin, dt_min;
  int newton_max_iter, boundary, max_levels, precision, order;
};

hipError_t launch_state_init(hipStream_t s, DevMesh& m, const double* d_prim, double gamma);
// rows [0, n) of a segment: U[i] from prim[perm[i]], R[i] = 0
hipError_t launch_state_init_rows(hipStream_t s, int n, const int* perm, const double* d_prim,
                                  double gamma, double* U, double* R);
hipError_t launch_dt(hipStream_t s, DevMesh& m, const StepArgs& a);
hipError_t launch_classify(hipStream_t s, DevMesh& m, const StepArgs& a);
// early_order: 1 or 2 marks the cells that apply their fluxes at their
// step's start (gather mode, one pass per face step) for that spatial order;
// 0 marks none
hipError_t launch_partitions(hipStream_t s, DevMesh& m, int early_order);
// r: the cells with tau_g <= tau_g of the tau_g list (a prefix); U: the cell
// states the pass reads (default: the mesh's U)
hipError_t launch_grad(hipStream_t s, DevMesh& m, const StepArgs& a, CellRange r, int tau_g,
                       const double* U = nullptr);
// optional flux features: feat bit 0 = gate statistics and face logging,
// bit 1 = learned guess (gamma = 1.4, gather mode)
// Faces whose fluxes the gradient launch computes (k_grad_flux): per chunk
// of kFuseChunk consecutive cells of the mesh order, the faces with both
// sides in the chunk and the chunk's boundary faces, as {face id, positions}
// with bits 0-7 the lower cell's index in the chunk, 8-9 its local face slot,
// 10-17 the higher cell's index, 18-19 its slot, bit 20 set for a boundary
// face.  Built at upload (gather mode, second order).
constexpr int kFuseChunk = 256;
// keys of the face list: (colour, tau_f) in colour mode; tau_f + 8 flocal
// while the chunk-local faces are kept apart (the faces between chunks
// first); tau_f else
inline int face_list_keys(const DevMesh& m) {
  if (m.scatter == TAFV_SCATTER_COLOUR) return m.ncolours * kMaxLevels;
  return m.split_local ? 2 * kMaxLevels : kMaxLevels;
}
struct LocalFaces {
  const int* start;  // [chunks + 1]
  const int2* face;  // [faces local to a chunk]
};

struct FluxFeatures {
  int feat = 0;
  const MlpDev* mlp = nullptr;
  float* log_rows = nullptr;
  unsigned long long* log_count = nullptr;
  long long log_cap = 0;
  double log_rate = 0.0;
  unsigned long long log_seed = 0, subit = 0;
  float guess_gate = 0.f;
  float guess_strength = 0.f;
};
// U: the cell states read at first order; Q: where gather mode stores the
// face fluxes (defaults: the mesh's U and Q); pass_mode and Qpred: the
// passes of the predictor/corrector form (see FluxArgs)
// dt_min_on_device: the kernels read dt_min from the device scalars (its
// bits in m.dscal[0]) instead of the host's value
// The faces are entries [first, first + count) and [first2, first2 + count2)
// of the face list.  key_max >= 0: those are the faces of key <= key_max
// (gather mode, one range from the list's start); when they are most of the
// faces the launch walks all faces in face order and takes those.
hipError_t launch_flux(hipStream_t s, DevMesh& m, const StepArgs& a, int first, int count,
                       const FluxFeatures& ft, const double* U = nullptr, void* Q = nullptr,
                       int pass_mode = 0, const void* Qpred = nullptr,
                       bool dt_min_on_device = false, int first2 = 0, int count2 = 0,
                       int key_max = -1);
// Gradient over the whole mesh (cells of tau_g <= tau_s) with the fluxes of
// the active faces local to a chunk (k_grad_flux); the other active faces are
// left to launch_flux.  Features: none, or the learned guess alone
// (ft.feat == 2, gamma 1.4); others give hipErrorInvalidValue.
hipError_t launch_grad_flux(hipStream_t s, DevMesh& m, const StepArgs& a, int tau_s,
                            const FluxFeatures& ft, bool dt_min_on_device);
// whether a gradient launch over `count` cells of the tau_g list takes the
// whole mesh in its own order (cells outside the key range skipped)
bool grad_whole_mesh(const DevMesh& m, int64_t count);
// the same for a flux launch over `count` faces
bool faces_whole_mesh(const DevMesh& m, int64_t count);
hipError_t launch_cell_gather(hipStream_t s, DevMesh& m, const ListRanges& r, int tau_s,
                              int tau_upd, double dt_min, int precision,
                              bool dt_min_on_device = false);
hipError_t launch_update(hipStream_t s, DevMesh& m, CellRange r, int tau_upd);
// the stages of a pipelined whole-mesh subiteration (gather mode, time
// order 1): gradients of the cells [c0, c1) of tau_g <= tau_s; fluxes of the
// faces [f0, f1) of tau_f <= tau_s in face order; the gather of the cells
// [c0, c1)
hipError_t launch_grad_chunk(hipStream_t s, DevMesh& m, const StepArgs& a, int tau_s, int c0,
                             int c1);
hipError_t launch_flux_chunk(hipStream_t s, DevMesh& m, const StepArgs& a,
                             const FluxFeatures& ft, int tau_s, int f0, int f1,
                             bool dt_min_on_device);
hipError_t launch_gather_chunk(hipStream_t s, DevMesh& m, int tau_s, int tau_upd, double dt_min,
                               int precision, int c0, int c1, bool dt_min_on_device);
// moving mesh: face volume rates sF from node velocities d_vel [n_nodes][3]
hipError_t launch_face_speed(hipStream_t s, DevMesh& m, const double* d_vel);
// one double per cell to the caller's order
hipError_t launch_vol_to_caller(hipStream_t s, DevMesh& m, const double* src, double* dst);
// predictor/corrector form (gather mode): predictions D of the cells whose
// step starts (tau <= tau_s) from the predictor fluxes Q0, and the states Ut
// at the end of subiteration `sub` of the cells that the passes over the
// faces of tau_f <= upd read (nkey <= upd); then the corrector sums
// of the first `count` listed cells for the faces whose step ends (tau_f <=
// tau_upd, Q holding phi0 + phi1), ending cells applied to U and Ut
hipError_t launch_predict(hipStream_t s, DevMesh& m, int tau_s, int sub, int upd,
                          double dt_min, int precision);
hipError_t launch_cell_gather2(hipStream_t s, DevMesh& m, CellRange r, int tau_upd,
                               double dt_min, int precision);
constexpr int kCellKeys = 2 * kMaxLevels;  // keys of the gather's cell list
// scalars 8, face starts kMaxKeys + 1, cell starts kMaxLevels + 1, gather-list
// starts kCellKeys + 1, the (tau_g, tau) histogram kMaxKeys
constexpr int kRbFace = 8, kRbCell = kRbFace + kMaxKeys + 1, kRbGather = kRbCell + kMaxLevels + 1,
              kRbHist = kRbGather + kCellKeys + 1, kReadbackInts = kRbHist + kMaxKeys;
// host-transfer staging: rows of 5 doubles or 1 byte, caller <-> internal order
hipError_t launch_to_caller_f64(hipStream_t s, DevMesh& m, const double* src, double* dst);
hipError_t launch_from_caller_f64(hipStream_t s, DevMesh& m, const double* src, double* dst);
hipError_t launch_to_caller_i8(hipStream_t s, DevMesh& m, const int8_t* src, int8_t* dst);
hipError_t launch_from_caller_i8(hipStream_t s, DevMesh& m, const int8_t* src, int8_t* dst);
// rows [0, n) of a segment to the caller's order: dst[perm[i]] = src[i]
hipError_t launch_rows_to_caller_f64(hipStream_t s, int n, const int* perm, const double* src,
                                    double* dst);
hipError_t launch_rows_to_caller_i8(hipStream_t s, int n, const int* perm, const int8_t* src,
                                   int8_t* dst);
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, unsigned long long v, int n);
hipError_t launch_fill_f64(hipStream_t s, double* p, double v, int64_t n);

// partition scratch sizes
int partition_blocks(int64_t n);

}  // namespace tafv
