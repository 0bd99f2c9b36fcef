/* Test driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only).  Reads a mesh, a primitive
 * state and node velocities from a raw file, runs the oracle in several
 * configurations and writes each final conserved state and two counters, so
 * that the test can compare them with the regular build.
 *
 * Input (native endianness): int64 n_nodes, n_tets; double xyz[n_nodes][3];
 * int64 tets[n_tets][4]; double prim[n_tets][5]; double vel[n_nodes][3].
 * Output, per configuration: double cons[n_tets][5]; int64 cell_updates,
 * newton_updates. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

typedef struct {
  int32_t order, time_order, boundary, max_levels, moving;
  int64_t n1, n2; /* two advance calls */
} config;

static const config kConfigs[] = {
    {1, 1, ORC_BC_WALL, 3, 0, 4, 3},     {2, 1, ORC_BC_WALL, 4, 0, 8, 5},
    {2, 1, ORC_BC_TRANSMIT, 3, 0, 6, 2}, {2, 2, ORC_BC_WALL, 3, 0, 8, 4},
    {2, 1, ORC_BC_WALL, 3, 1, 6, 2},
};

static void* read_n(FILE* f, size_t size, size_t n) {
  void* p = malloc(size * (n ? n : 1));
  if (!p || fread(p, size, n, f) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: oracle_check INPUT OUTPUT\n");
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t* hdr = (int64_t*)read_n(in, sizeof(int64_t), 2);
  const int64_t nn = hdr[0], nt = hdr[1];
  double* xyz = (double*)read_n(in, sizeof(double), (size_t)(3 * nn));
  int64_t* tets = (int64_t*)read_n(in, sizeof(int64_t), (size_t)(4 * nt));
  double* prim = (double*)read_n(in, sizeof(double), (size_t)(5 * nt));
  double* vel = (double*)read_n(in, sizeof(double), (size_t)(3 * nn));
  fclose(in);
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  orc_mesh* m = NULL;
  if (orc_mesh_build(nn, xyz, nt, tets, &m) != ORC_OK) return 3;
  double* cons = (double*)malloc(sizeof(double) * 5 * (size_t)nt);
  for (size_t k = 0; k < sizeof(kConfigs) / sizeof(kConfigs[0]); ++k) {
    const config* c = &kConfigs[k];
    orc_params p = {1.4, 0.5, 1e-12, 1e-9, c->max_levels, c->order, 50, c->boundary, 1,
                    c->time_order};
    orc_state* s = NULL;
    if (orc_state_new(m, &p, prim, &s) != ORC_OK) return 4;
    if (c->moving && orc_state_motion(s, vel) != ORC_OK) return 5;
    if (orc_advance(s, c->n1) != ORC_OK || orc_advance(s, c->n2) != ORC_OK) return 6;
    orc_stats st;
    if (orc_state_read(s, cons, NULL, NULL) != ORC_OK || orc_state_stats(s, &st) != ORC_OK)
      return 7;
    fwrite(cons, sizeof(double), 5 * (size_t)nt, out);
    fwrite(&st.cell_updates, sizeof(int64_t), 1, out);
    fwrite(&st.newton_updates, sizeof(int64_t), 1, out);
    orc_state_free(s);
  }
  orc_mesh_free(m);
  fclose(out);
  free(cons);
  free(hdr);
  free(xyz);
  free(tets);
  free(prim);
  free(vel);
  return 0;
}
