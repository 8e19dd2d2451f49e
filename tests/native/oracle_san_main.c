/* Host sanitizer run of the oracle's C integrals (AddressSanitizer and
 * UndefinedBehaviorSanitizer): reads one basis, density and energy-weighted
 * density from a flat input file, calls every entry point of the oracle's
 * integral library once and writes the results, in call order, to the
 * output file, so that the test compares them with the library as the
 * oracle loads it.  Test infrastructure only.
 *
 * Input (native endianness): int32 nsh, nbf, natom, nprim_total; int32
 * l, atom, nprim, pofs, bf [nsh]; int32 Z [natom]; float64 exps, coefs
 * [nprim_total]; float64 xyz [natom][3]; float64 P, W [nbf][nbf]. */
#include <stdio.h>
#include <stdlib.h>

void or_boys(int mmax, double T, double *F);
void or_one_electron(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                     const int *pofs, const int *bf, const double *exps, const double *coefs,
                     int natom, const double *xyz, const int *Z, double *S, double *T,
                     double *V);
void or_eri_quartet(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                    const int *pofs, const int *bf, const double *exps, const double *coefs,
                    const double *xyz, int a, int b, int c, int d, double *out, double *deriv);
void or_eri_tensor(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                   const int *pofs, const int *bf, const double *exps, const double *coefs,
                   const double *xyz, double *out);
void or_schwarz(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                const int *pofs, const int *bf, const double *exps, const double *coefs,
                const double *xyz, double *Q);
long or_jk(int nsh, int nbf, const int *l, const int *atom, const int *nprim, const int *pofs,
           const int *bf, const double *exps, const double *coefs, const double *xyz,
           const double *Q, double tau, const double *P, double *J, double *K);
long or_jk_sample(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                  const int *pofs, const int *bf, const double *exps, const double *coefs,
                  const double *xyz, const double *Q, double tau, const double *P, int stride,
                  int nthreads, double *J, double *K);
long or_grad_2e_kx(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                   const int *pofs, const int *bf, const double *exps, const double *coefs,
                   const double *xyz, int natom, const double *Q, double tau, const double *P,
                   double kx, double *g);
long or_grad_2e_atoms(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                      const int *pofs, const int *bf, const double *exps, const double *coefs,
                      const double *xyz, int natom, const double *Q, double tau, const double *P,
                      const int *amask, double *g);
void or_grad_1e(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                const int *pofs, const int *bf, const double *exps, const double *coefs,
                int natom, const double *xyz, const int *Z, const double *P, const double *W,
                double *g);
void or_grad_1e_atoms(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                      const int *pofs, const int *bf, const double *exps, const double *coefs,
                      int natom, const double *xyz, const int *Z, const double *P,
                      const double *W, const int *amask, double *g);
void or_jk_pairs(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                 const int *pofs, const int *bf, const double *exps, const double *coefs,
                 const double *xyz, const double *Q, double tau, const double *P, int npairs,
                 const int *pa, const int *pb, double *J, double *K);

static void *take(FILE *f, size_t n, size_t sz) {
  void *p = calloc(n ? n : 1, sz);
  if (!p || fread(p, sz, n, f) != n) {
    fprintf(stderr, "input: short read\n");
    exit(2);
  }
  return p;
}

static void emit(FILE *f, const double *x, size_t n) {
  if (fwrite(x, sizeof(double), n, f) != n) {
    fprintf(stderr, "output: short write\n");
    exit(2);
  }
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE *in = fopen(argv[1], "rb");
  if (!in) return 2;
  int *head = take(in, 4, sizeof(int));
  const int nsh = head[0], nbf = head[1], nat = head[2], npt = head[3];
  int *l = take(in, nsh, sizeof(int)), *atom = take(in, nsh, sizeof(int));
  int *nprim = take(in, nsh, sizeof(int)), *pofs = take(in, nsh, sizeof(int));
  int *bf = take(in, nsh, sizeof(int)), *Z = take(in, nat, sizeof(int));
  double *exps = take(in, npt, sizeof(double)), *coefs = take(in, npt, sizeof(double));
  double *xyz = take(in, 3 * (size_t)nat, sizeof(double));
  const size_t nn = (size_t)nbf * nbf;
  double *P = take(in, nn, sizeof(double)), *W = take(in, nn, sizeof(double));
  fclose(in);
  FILE *out = fopen(argv[2], "wb");
  if (!out) return 2;

  double F[17];
  for (int k = 0; k < 64; ++k) {
    or_boys(16, 0.37 * k * k / 8.0, F);
    emit(out, F, 17);
  }
  double *S = calloc(nn, 8), *T = calloc(nn, 8), *V = calloc(nn, 8);
  or_one_electron(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, nat, xyz, Z, S, T, V);
  emit(out, S, nn);
  emit(out, T, nn);
  emit(out, V, nn);
  double *eri = calloc(nn * nn, 8);
  or_eri_tensor(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, eri);
  emit(out, eri, nn * nn);
  /* the last shell with itself and the first two: the highest angular
   * momentum block and its centre derivatives */
  const int a = nsh - 1, c0 = 0, c1 = nsh > 1 ? 1 : 0;
  const int na = (l[a] + 1) * (l[a] + 2) / 2, n0 = (l[c0] + 1) * (l[c0] + 2) / 2,
            n1 = (l[c1] + 1) * (l[c1] + 2) / 2;
  const size_t nq = (size_t)na * na * n0 * n1;
  double *blk = calloc(nq, 8), *der = calloc(12 * nq, 8);
  or_eri_quartet(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, a, a, c0, c1, blk, der);
  emit(out, blk, nq);
  emit(out, der, 12 * nq);
  double *Q = calloc((size_t)nsh * nsh, 8);
  or_schwarz(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, Q);
  emit(out, Q, (size_t)nsh * nsh);
  double *J = calloc(nn, 8), *K = calloc(nn, 8);
  double cnt = (double)or_jk(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, Q, 1e-12, P, J, K);
  emit(out, &cnt, 1);
  emit(out, J, nn);
  emit(out, K, nn);
  double *Js = calloc(nn, 8), *Ks = calloc(nn, 8);
  cnt = (double)or_jk_sample(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, Q, 1e-12, P,
                             3, 2, Js, Ks);
  emit(out, &cnt, 1);
  emit(out, Js, nn);
  emit(out, Ks, nn);
  const int npairs = nsh * (nsh + 1) / 2;
  int *pa = calloc(npairs, sizeof(int)), *pb = calloc(npairs, sizeof(int));
  for (int i = 0, k = 0; i < nsh; ++i)
    for (int j = 0; j <= i; ++j, ++k) {
      pa[k] = i;
      pb[k] = j;
    }
  double *Jp = calloc(nn, 8), *Kp = calloc(nn, 8);
  or_jk_pairs(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, Q, 1e-12, P, npairs, pa, pb,
              Jp, Kp);
  emit(out, Jp, nn);
  emit(out, Kp, nn);
  double *g = calloc(3 * (size_t)nat, 8);
  or_grad_2e_kx(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, nat, Q, 1e-12, P, 0.2, g);
  emit(out, g, 3 * (size_t)nat);
  int *amask = calloc(nat, sizeof(int));
  for (int i = 0; i < nat; i += 2) amask[i] = 1;
  double *ga = calloc(3 * (size_t)nat, 8);
  or_grad_2e_atoms(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, nat, Q, 1e-12, P, amask, ga);
  emit(out, ga, 3 * (size_t)nat);
  double *g1 = calloc(3 * (size_t)nat, 8), *g1a = calloc(3 * (size_t)nat, 8);
  or_grad_1e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, nat, xyz, Z, P, W, g1);
  or_grad_1e_atoms(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, nat, xyz, Z, P, W, amask, g1a);
  emit(out, g1, 3 * (size_t)nat);
  emit(out, g1a, 3 * (size_t)nat);
  if (fclose(out) != 0) return 2;

  free(head), free(l), free(atom), free(nprim), free(pofs), free(bf), free(Z);
  free(exps), free(coefs), free(xyz), free(P), free(W), free(S), free(T), free(V), free(eri);
  free(blk), free(der), free(Q), free(J), free(K), free(Js), free(Ks), free(pa), free(pb);
  free(Jp), free(Kp), free(g), free(amask), free(ga), free(g1), free(g1a);
  return 0;
}
