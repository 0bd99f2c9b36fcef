// Test driver for a sanitizer build of the library's host mesh preparation
// (AddressSanitizer and UndefinedBehaviorSanitizer, host code only).  Reads
// a mesh from a raw file (the layout of oracle_check.c's input), prepares it
// in the four orders (faces colour-major or not, cells Morton or not) and
// writes, for the colour-major caller-order preparation, what the library's
// tafv_mesh_inspect reports: face, boundary and colour counts, the face
// colours, area vectors and the cell neighbours.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "tafv_internal.h"

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: mesh_prep_check INPUT OUTPUT\n");
    return 2;
  }
  std::FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t hdr[2];
  if (std::fread(hdr, sizeof(int64_t), 2, in) != 2) return 2;
  std::vector<double> xyz(3 * hdr[0]);
  std::vector<int64_t> tets(4 * hdr[1]);
  if (std::fread(xyz.data(), sizeof(double), xyz.size(), in) != xyz.size() ||
      std::fread(tets.data(), sizeof(int64_t), tets.size(), in) != tets.size())
    return 2;
  std::fclose(in);
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  for (int order = 0; order < 4; ++order) {
    const bool colour_major = !(order & 1), morton = (order & 2) != 0;
    tafv::HostMesh hm;
    std::string err;
    if (tafv::build_host_mesh(hdr[0], xyz.data(), hdr[1], tets.data(), colour_major, morton,
                              &hm, &err) != TAFV_OK) {
      std::fprintf(stderr, "%s\n", err.c_str());
      return 3;
    }
    if (order != 0) continue;
    const int64_t counts[3] = {hm.nf, hm.nbnd, hm.ncolours};
    std::fwrite(counts, sizeof(int64_t), 3, out);
    std::fwrite(hm.fcol.data(), sizeof(int8_t), hm.fcol.size(), out);
    // area vectors as [nf][3], neighbours as [nc][4] (the inspect layout)
    for (int64_t f = 0; f < hm.nf; ++f)
      for (int q = 0; q < 3; ++q) std::fwrite(&hm.fA[q * hm.nf + f], sizeof(double), 1, out);
    for (int64_t i = 0; i < hm.nc; ++i)
      for (int m = 0; m < 4; ++m) std::fwrite(&hm.nb[m * hm.nc + i], sizeof(int32_t), 1, out);
  }
  std::fclose(out);
  return 0;
}
