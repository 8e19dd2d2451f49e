/* Host sanitizer run of the library: libbeadscf built with its host code
 * (the batch set-up, screening and work lists, grid chunking, SCF control,
 * integrators, checkpoints and the C ABI) under AddressSanitizer and
 * UndefinedBehaviorSanitizer, driven through the C ABI over one ring
 * polymer: SCF at both precisions and with the learned guess, forces, MD
 * steps, a checkpoint written and read back, B3LYP energies and forces and
 * a string-method step, then the rejection of bad calls.  Device code is
 * built as usual.  Test infrastructure only.
 *
 * usage: engine_san basis.json geometry.txt checkpoint-path
 * geometry.txt: "P N", N atomic numbers, then P x N x 3 coordinates (bohr). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "beadscf.h"

static int fails = 0;

static void check(bscf_status rc, const char* what) {
  printf("%-28s %s\n", what, rc == BSCF_OK ? "ok" : bscf_last_error());
  fflush(stdout);
  if (rc != BSCF_OK) ++fails;
}

static void refused(bscf_status rc, const char* what) {
  printf("%-28s %s\n", what, rc != BSCF_OK ? "refused" : "ACCEPTED");
  fflush(stdout);
  if (rc == BSCF_OK) ++fails;
}

static char* slurp(const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  const long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* s = malloc(n + 1);
  if (s && fread(s, 1, n, f) != (size_t)n) {
    free(s);
    s = NULL;
  }
  if (s) s[n] = 0;
  fclose(f);
  return s;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s basis.json geometry.txt checkpoint\n", argv[0]);
    return 2;
  }
  char* basis = slurp(argv[1]);
  FILE* g = fopen(argv[2], "r");
  int P = 0, N = 0;
  if (!basis || !g || fscanf(g, "%d %d", &P, &N) != 2 || P < 2 || N < 1) return 2;
  int* Z = malloc(sizeof(int) * P * N);
  int* nat = malloc(sizeof(int) * P);
  int* chg = calloc(P, sizeof(int));
  double* x = malloc(sizeof(double) * 3 * P * N);
  for (int a = 0; a < N; ++a)
    if (fscanf(g, "%d", &Z[a]) != 1) return 2;
  for (int j = 0; j < P; ++j) {
    nat[j] = N;
    memcpy(Z + j * N, Z, sizeof(int) * N);
  }
  for (int k = 0; k < 3 * P * N; ++k)
    if (fscanf(g, "%lf", &x[k]) != 1) return 2;
  fclose(g);
  double* m = malloc(sizeof(double) * N);
  for (int a = 0; a < N; ++a) m[a] = Z[a] == 1 ? 1837.4 : 29156.9;
  double* E = malloc(sizeof(double) * P);
  double* F = malloc(sizeof(double) * 3 * P * N);
  int* it = malloc(sizeof(int) * P);
  int* st = malloc(sizeof(int) * P);

  bscf_ctx* c = NULL;
  check(bscf_create(0, NULL, &c), "create");
  if (!c) return 1;
  check(bscf_load_basis(c, basis), "load_basis");
  check(bscf_set_instances(c, P, nat, Z, chg), "set_instances");
  check(bscf_set_geometries(c, x), "set_geometries");
  bscf_scf_opts o;
  bscf_default_opts(&o);
  check(bscf_run_scf(c, &o, E, it, st), "scf fp64");
  check(bscf_forces(c, F), "forces");
  o.precision = BSCF_MIXED;
  o.guess = BSCF_GUESS_PREVIOUS;
  check(bscf_run_scf(c, &o, E, it, st), "scf mixed");
  o.density = BSCF_DENSITY_EIG;
  o.graph = 0;
  o.incremental = 0;
  check(bscf_run_scf(c, &o, E, it, st), "scf eig, full builds");
  bscf_default_opts(&o);
  o.guess = BSCF_GUESS_LEARNED;
  bscf_pimd_opts po;
  bscf_pimd_default_opts(&po);
  check(bscf_pimd_init(c, &po, m, NULL), "pimd_init");
  for (int s = 0; s < 3; ++s) {
    check(bscf_pimd_step(c, &o, E, it, st, F), "pimd_step (learned guess)");
    float loss = 0.f;
    check(bscf_guess_train(c, 20, &loss), "guess_train");
  }
  check(bscf_checkpoint_save(c, argv[3]), "checkpoint_save");
  check(bscf_checkpoint_load(c, argv[3]), "checkpoint_load");
  o.guess = BSCF_GUESS_EXTRAPOLATED;
  o.deterministic = 1;
  check(bscf_pimd_step(c, &o, E, it, st, F), "pimd_step (extrapolated)");
  double obs[3];
  check(bscf_pimd_state(c, NULL, NULL, obs), "pimd_state");
  check(bscf_set_xc(c, 1), "set_xc b3lyp");
  bscf_default_opts(&o);
  check(bscf_run_scf(c, &o, E, it, st), "scf b3lyp");
  check(bscf_forces(c, F), "forces b3lyp");
  check(bscf_set_xc(c, 0), "set_xc hf");
  bscf_string_opts so;
  bscf_string_default_opts(&so);
  check(bscf_string_init(c, &so), "string_init");
  check(bscf_string_step(c, &o, E, it, st, F), "string_step");
  static char buf[1 << 16];
  check(bscf_get_stats(c, buf, sizeof buf), "get_stats");

  refused(bscf_load_basis(c, "{\"not a basis\": 1"), "bad basis json");
  x[0] = 0.0 / 0.0;
  refused(bscf_set_geometries(c, x), "non-finite geometry");
  refused(bscf_checkpoint_load(c, argv[1]), "foreign checkpoint");
  int one = 1;
  refused(bscf_set_instances(c, 1, &one, &one, chg), "odd electron count");

  check(bscf_destroy(c), "destroy");
  free(basis), free(Z), free(nat), free(chg), free(x), free(m), free(E), free(F), free(it),
      free(st);
  printf("failures %d\n", fails);
  return fails ? 1 : 0;
}
