// Host mesh preprocessing: faces of a tetrahedral mesh, FP64 geometry, a
// face colouring for the atomic-free scatter, and least-squares weights.
//
// Finite volumes (Sec. 2.1, Eq. (1)) need per cell its volume and the outward
// area vectors of its faces; the MUSCL reconstruction needs, per cell, the
// weighted least-squares gradient operator over its 4 face neighbours and
// the offsets from the cell centroid to its face centroids.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "tafv_internal.h"

namespace tafv {
namespace {

struct FaceRec {
  int64_t v[3];
  int32_t cell;
  int32_t slot;
};

inline bool rec_less(const FaceRec& x, const FaceRec& y) {
  if (x.v[0] != y.v[0]) return x.v[0] < y.v[0];
  if (x.v[1] != y.v[1]) return x.v[1] < y.v[1];
  if (x.v[2] != y.v[2]) return x.v[2] < y.v[2];
  return x.cell < y.cell;
}

inline bool same_key(const FaceRec& x, const FaceRec& y) {
  return x.v[0] == y.v[0] && x.v[1] == y.v[1] && x.v[2] == y.v[2];
}

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

}  // namespace

tafv_status build_host_mesh(int64_t n_nodes, const double* xyz, int64_t n_tets,
                            const int64_t* tets, bool colour_major, bool morton,
                            HostMesh* out, std::string* err) {
  if (n_tets >= (int64_t(1) << 29)) {
    *err = "mesh too large: at most 2^29 tets";
    return TAFV_E_ARG;
  }
  if (n_nodes >= (int64_t(1) << 31)) {
    *err = "mesh too large: at most 2^31 - 1 nodes";
    return TAFV_E_ARG;
  }
  const int64_t nc = n_tets;
  auto node = [&](int64_t id) { return V3{xyz[3 * id], xyz[3 * id + 1], xyz[3 * id + 2]}; };
  // validate and measure in the caller's order
  std::vector<V3> xcc(nc);
  std::vector<double> volc(nc);
  for (int64_t t = 0; t < nc; ++t) {
    const int64_t* v = tets + 4 * t;
    for (int k = 0; k < 4; ++k) {
      if (v[k] < 0 || v[k] >= n_nodes) {
        *err = "tet " + std::to_string(t) + ": node id out of range";
        return TAFV_E_MESH;
      }
    }
    V3 p0 = node(v[0]), p1 = node(v[1]), p2 = node(v[2]), p3 = node(v[3]);
    double det = dot(sub(p1, p0), cross(sub(p2, p0), sub(p3, p0)));
    if (!(det > 0.0)) {
      *err = "tet " + std::to_string(t) + ": non-positive volume (tets must be positively oriented)";
      return TAFV_E_MESH;
    }
    volc[t] = det / 6.0;
    xcc[t] = {(p0.x + p1.x + p2.x + p3.x) * 0.25, (p0.y + p1.y + p2.y + p3.y) * 0.25,
              (p0.z + p1.z + p2.z + p3.z) * 0.25};
  }
  // internal cell order: the caller's, or the Morton (Z-order) code of the
  // centroid in the bounding box, 21 bits per axis, ties by caller id
  out->perm.resize(nc);
  std::iota(out->perm.begin(), out->perm.end(), 0);
  if (morton) {
    V3 lo = xcc[0], hi = xcc[0];
    for (const V3& c : xcc) {
      lo = {std::min(lo.x, c.x), std::min(lo.y, c.y), std::min(lo.z, c.z)};
      hi = {std::max(hi.x, c.x), std::max(hi.y, c.y), std::max(hi.z, c.z)};
    }
    auto spread = [](uint64_t v) {  // bits 0..20 -> every third bit
      v &= 0x1fffff;
      v = (v | v << 32) & 0x1f00000000ffffull;
      v = (v | v << 16) & 0x1f0000ff0000ffull;
      v = (v | v << 8) & 0x100f00f00f00f00full;
      v = (v | v << 4) & 0x10c30c30c30c30c3ull;
      v = (v | v << 2) & 0x1249249249249249ull;
      return v;
    };
    auto q = [](double x, double a, double b) {
      double s = b > a ? (x - a) / (b - a) : 0.0;
      return (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(s * 2097151.0)));
    };
    std::vector<uint64_t> key(nc);
    for (int64_t t = 0; t < nc; ++t)
      key[t] = spread(q(xcc[t].x, lo.x, hi.x)) | spread(q(xcc[t].y, lo.y, hi.y)) << 1 |
               spread(q(xcc[t].z, lo.z, hi.z)) << 2;
    std::stable_sort(out->perm.begin(), out->perm.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  }
  std::vector<int32_t> inv(nc);
  for (int64_t i = 0; i < nc; ++i) inv[out->perm[i]] = (int32_t)i;
  std::vector<V3> xc(nc);
  out->vol.resize(nc);
  for (int64_t i = 0; i < nc; ++i) {
    xc[i] = xcc[out->perm[i]];
    out->vol[i] = volc[out->perm[i]];
  }
  std::vector<FaceRec> rec(4 * nc);
  for (int64_t t = 0; t < nc; ++t) {
    const int64_t* v = tets + 4 * t;
    for (int s = 0; s < 4; ++s) {
      FaceRec& r = rec[4 * t + s];
      int q = 0;
      for (int k = 0; k < 4; ++k)
        if (k != s) r.v[q++] = v[k];
      std::sort(r.v, r.v + 3);
      r.cell = inv[t];
      r.slot = s;
    }
  }
  // order by (sorted vertex triple, cell): a counting sort on the lowest
  // vertex id, then a comparison sort inside each (small) bucket
  {
    std::vector<int64_t> bstart(n_nodes + 1, 0);
    for (const FaceRec& r : rec) ++bstart[r.v[0] + 1];
    for (int64_t v = 0; v < n_nodes; ++v) bstart[v + 1] += bstart[v];
    std::vector<FaceRec> sorted(rec.size());
    std::vector<int64_t> cur(bstart.begin(), bstart.end() - 1);
    for (const FaceRec& r : rec) sorted[cur[r.v[0]]++] = r;
    for (int64_t v = 0; v < n_nodes; ++v)
      if (bstart[v + 1] - bstart[v] > 1)
        std::sort(sorted.begin() + bstart[v], sorted.begin() + bstart[v + 1], rec_less);
    rec.swap(sorted);
  }

  // faces in key order: lower cell = L
  struct RawFace {
    int32_t L, R;
    int8_t sL, sR;
    int32_t v[3];
    V3 A, xf;
  };
  std::vector<RawFace> faces;
  faces.reserve(2 * nc + nc / 2);
  int64_t nb = 0;
  for (size_t i = 0; i < rec.size();) {
    size_t j = i + 1;
    while (j < rec.size() && same_key(rec[j], rec[i])) ++j;
    if (j - i > 2 || (j - i == 2 && rec[i].cell == rec[i + 1].cell)) {
      *err = "a face is shared by more than two tets (cell " + std::to_string(rec[i].cell) + ")";
      return TAFV_E_MESH;
    }
    RawFace f;
    f.L = rec[i].cell;
    f.sL = (int8_t)rec[i].slot;
    for (int k = 0; k < 3; ++k) f.v[k] = (int32_t)rec[i].v[k];
    if (j - i == 2) {
      f.R = rec[i + 1].cell;
      f.sR = (int8_t)rec[i + 1].slot;
    } else {
      f.R = -1;
      f.sR = -1;
      ++nb;
    }
    V3 a = node(rec[i].v[0]), b = node(rec[i].v[1]), c = node(rec[i].v[2]);
    V3 n = cross(sub(b, a), sub(c, a));
    f.A = {0.5 * n.x, 0.5 * n.y, 0.5 * n.z};
    f.xf = {(a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0, (a.z + b.z + c.z) / 3.0};
    if (dot(f.A, sub(f.xf, xc[f.L])) < 0.0) f.A = {-f.A.x, -f.A.y, -f.A.z};
    faces.push_back(f);
    i = j;
  }
  rec.clear();
  rec.shrink_to_fit();
  const int64_t nf = (int64_t)faces.size();

  // greedy colouring: faces visited by (L, R); a face takes the lowest
  // colour not yet used by another face of either cell
  // (a stable order by (L, R): counting sort on L, then a stable insertion
  // sort on R among the at most 4 faces of each L)
  std::vector<int32_t> order(nf);
  {
    std::vector<int64_t> lstart(nc + 1, 0);
    for (int64_t f = 0; f < nf; ++f) ++lstart[faces[f].L + 1];
    for (int64_t i = 0; i < nc; ++i) lstart[i + 1] += lstart[i];
    std::vector<int64_t> cur(lstart.begin(), lstart.end() - 1);
    for (int64_t f = 0; f < nf; ++f) order[cur[faces[f].L]++] = (int32_t)f;
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t a = lstart[i] + 1; a < lstart[i + 1]; ++a) {
        int32_t x = order[a];
        int64_t b = a;
        while (b > lstart[i] && faces[order[b - 1]].R > faces[x].R) {
          order[b] = order[b - 1];
          --b;
        }
        order[b] = x;
      }
  }
  std::vector<uint8_t> used(nc, 0);
  std::vector<int8_t> colour(nf);
  int ncol = 0;
  for (int32_t f : order) {
    unsigned m = used[faces[f].L];
    if (faces[f].R >= 0) m |= used[faces[f].R];
    int c = 0;
    while (m & (1u << c)) ++c;
    if (c >= kMaxColours) {
      *err = "face colouring needs more than 8 colours";
      return TAFV_E_MESH;
    }
    colour[f] = (int8_t)c;
    used[faces[f].L] |= (uint8_t)(1u << c);
    if (faces[f].R >= 0) used[faces[f].R] |= (uint8_t)(1u << c);
    ncol = std::max(ncol, c + 1);
  }
  // final face order: by colour, then by (L, R) within the colour
  if (colour_major)
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return colour[x] < colour[y]; });

  out->nc = nc;
  out->nf = nf;
  out->nbnd = nb;
  out->ncolours = ncol;
  out->fhL.resize(nf);
  out->fhR.resize(nf);
  out->fcol.resize(nf);
  out->fA.resize(3 * nf);
  out->fnode.resize(3 * nf);
  out->n_nodes = n_nodes;
  out->nb.assign(4 * nc, 0);
  out->c2f.assign(4 * nc, 0);
  std::vector<V3> xf_new(nf);
  for (int c = 0; c <= kMaxColours; ++c) out->colour_start[c] = nf;
  for (int64_t k = nf - 1; k >= 0; --k) out->colour_start[colour[order[k]]] = k;
  for (int c = kMaxColours - 1; c >= 0; --c)
    if (out->colour_start[c] > out->colour_start[c + 1]) out->colour_start[c] = out->colour_start[c + 1];
  for (int64_t k = 0; k < nf; ++k) {
    const RawFace& f = faces[order[k]];
    out->fhL[k] = 4 * f.L + f.sL;
    out->fhR[k] = f.R >= 0 ? 4 * f.R + f.sR : -1;
    out->fcol[k] = colour[order[k]];
    out->fA[k] = f.A.x;
    out->fA[nf + k] = f.A.y;
    out->fA[2 * nf + k] = f.A.z;
    for (int q = 0; q < 3; ++q) out->fnode[q * nf + k] = f.v[q];
    xf_new[k] = f.xf;
    out->c2f[f.sL * nc + f.L] = (int32_t)k;
    out->nb[f.sL * nc + f.L] = f.R >= 0 ? f.R : -(int32_t)(k + 1);
    if (f.R >= 0) {
      out->c2f[f.sR * nc + f.R] = (int32_t)k;
      out->nb[f.sR * nc + f.R] = f.L;
    }
  }

  // least squares: neighbour (or mirror ghost) offsets d_m, weights
  // 1/|d_m|^2, M = sum w d d^T, coefficient vectors c_j = M^-1 w_j d_j.
  // The gradient is only used through its change to the face centroids,
  // G . r_m = sum_j (c_j . r_m) (W_j - W_i), r_m = x_f(m) - x_i, so the
  // coefficients stored are c_j . r_m; the 4 offsets of a tetrahedron sum
  // to zero (each vertex is in 3 of its faces), so m = 3 follows from the
  // others and only m < 3 is stored.
  out->grc.assign(12 * nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    V3 d[4], rm[4];
    double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int m = 0; m < 4; ++m) {
      int32_t f = out->c2f[m * nc + i];
      int32_t other = out->nb[m * nc + i];
      V3 r = sub(xf_new[f], xc[i]);
      rm[m] = r;
      if (other >= 0) {
        d[m] = sub(xc[other], xc[i]);
      } else {
        V3 A = {out->fA[f], out->fA[nf + f], out->fA[2 * nf + f]};
        double an = std::sqrt(dot(A, A));
        V3 n = {A.x / an, A.y / an, A.z / an};
        double h = 2.0 * dot(r, n);  // ghost = centroid mirrored in the face plane
        d[m] = {h * n.x, h * n.y, h * n.z};
      }
      double w = 1.0 / dot(d[m], d[m]);
      double dv[3] = {d[m].x, d[m].y, d[m].z};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] += w * dv[a] * dv[b];
    }
    double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    if (!(std::fabs(det) > 0.0)) {
      *err = "singular least-squares matrix at cell " + std::to_string(i);
      return TAFV_E_MESH;
    }
    double inv[3][3];
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
    inv[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    inv[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    inv[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
    inv[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    inv[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    V3 c[4];
    for (int j = 0; j < 4; ++j) {
      double w = 1.0 / dot(d[j], d[j]);
      double dv[3] = {w * d[j].x, w * d[j].y, w * d[j].z};
      double cv[3];
      for (int a = 0; a < 3; ++a) cv[a] = inv[a][0] * dv[0] + inv[a][1] * dv[1] + inv[a][2] * dv[2];
      c[j] = {cv[0], cv[1], cv[2]};
    }
    for (int m = 0; m < 3; ++m)
      for (int j = 0; j < 4; ++j) out->grc[(4 * m + j) * nc + i] = dot(c[j], rm[m]);
  }
  return TAFV_OK;
}

}  // namespace tafv
