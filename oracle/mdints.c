/*
 * Plain FP64 CPU oracle for closed-shell Hartree-Fock integrals, J/K and
 * energy gradients.  TEST INFRASTRUCTURE ONLY: it exists to check the HIP
 * path and shares no code with it.
 *
 * The paper fixes the level of theory only by name (Gaussian-basis SCF with
 * analytic BO forces, an integral cutoff of 1e-12; Section 3.1).  Everything
 * here is the textbook definition, written out:
 *   - McMurchie-Davidson Hermite expansion of Gaussian overlap distributions
 *     (Helgaker, Jorgensen and Olsen, "Molecular Electronic-Structure
 *     Theory", Sections 9.5-9.9): overlap via E^{ij}_0, nuclear attraction and
 *     electron repulsion via the Hermite Coulomb integrals R_{tuv}.
 *   - Kinetic energy from the second derivative of the ket Gaussian.
 *   - Derivatives of a Cartesian Gaussian with respect to its centre:
 *     d/dA_x g(l_x) = 2 alpha g(l_x + 1) - l_x g(l_x - 1).
 *   - Operator-centre derivative of the nuclear attraction via
 *     dR_{tuv}/dC_x = -R_{t+1,u,v}.
 *   - J_mn = sum_ls (mn|ls) P_ls and K_ml = sum_ns (mn|ls) P_ns summed over all
 *     ordered index quartets; each canonical shell quartet contributes once
 *     for each of its distinct shell permutations.
 *   - Schwarz screening: a canonical shell quartet is skipped when
 *     Q_ab Q_cd < tau, Q_ab = sqrt(max |(mn|mn)|) over the pair's functions.
 * The Boys function is evaluated by its power series (in long double) and,
 * for large T, from erf plus upward recursion.
 *
 * Basis functions are contracted Cartesian Gaussians; shell functions are
 * ordered lexicographically (x before y before z; xx,xy,xz,yy,yz,zz for d).
 * The coefficient array holds d_k times the radial primitive normalisation and
 * the contraction renormalisation; the per-component factor
 * 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!) is applied here.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LMAX 3          /* highest shell l after raising by one (d+1 = f) */
#define LTOT (4 * LMAX + 2)
#define NE (LMAX + 4)   /* index range of E tables per side (kinetic derivative needs l+4) */
#define NT (2 * LMAX + 6)

typedef struct {
  int nsh, nbf;
  const int *l, *atom, *nprim, *pofs, *bf;
  const double *exps, *coefs, *xyz; /* xyz: per atom */
} basis_t;

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents of component c of a shell with angular momentum l. */
static void cart(int l, int c, int *lx, int *ly, int *lz) {
  int n = 0;
  for (int x = l; x >= 0; --x)
    for (int y = l - x; y >= 0; --y) {
      if (n == c) { *lx = x; *ly = y; *lz = l - x - y; return; }
      ++n;
    }
}

static double dfact(int n) { /* n!! with (-1)!! = 1 */
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

static double comp_norm(int lx, int ly, int lz) {
  return 1.0 / sqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
}

/* ---------------------------------------------------------------- Boys F_m(T) */
/* F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, m = 0..mmax. */
void or_boys(int mmax, double T, double *F) {
  if (T < 30.0) {
    /* F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) */
    long double term = 1.0L / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 1000; ++k) {
      term *= (2.0L * T) / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < 1e-22L * sum) break;
    }
    long double eT = expl(-(long double)T);
    long double f = eT * sum;
    F[mmax] = (double)f;
    /* downward: F_m = (2T F_{m+1} + exp(-T)) / (2m+1) */
    for (int m = mmax - 1; m >= 0; --m) {
      f = (2.0L * T * f + eT) / (2 * m + 1);
      F[m] = (double)f;
    }
  } else {
    double eT = exp(-T);
    double f = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
    F[0] = f;
    /* upward: F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T) */
    for (int m = 0; m < mmax; ++m) {
      f = ((2 * m + 1) * f - eT) / (2.0 * T);
      F[m + 1] = f;
    }
  }
}

/* ------------------------------------------------- Hermite expansion E^{ij}_t */
/* One Cartesian direction; XAB = A - B.  E[i][j][t], i<=imax, j<=jmax. */
static void hermite_E(int imax, int jmax, double a, double b, double XAB,
                      double E[NE][NE][NT]) {
  double p = a + b, mu = a * b / p;
  double XPA = -b / p * XAB, XPB = a / p * XAB, h = 0.5 / p;
  memset(E, 0, sizeof(double) * NE * NE * NT);
  E[0][0][0] = exp(-mu * XAB * XAB);
  for (int i = 0; i <= imax; ++i) {
    if (i > 0)
      for (int t = 0; t <= i; ++t) {
        double v = XPA * E[i - 1][0][t] + (t + 1) * E[i - 1][0][t + 1];
        if (t > 0) v += h * E[i - 1][0][t - 1];
        E[i][0][t] = v;
      }
    for (int j = 1; j <= jmax; ++j)
      for (int t = 0; t <= i + j; ++t) {
        double v = XPB * E[i][j - 1][t] + (t + 1) * E[i][j - 1][t + 1];
        if (t > 0) v += h * E[i][j - 1][t - 1];
        E[i][j][t] = v;
      }
  }
}

/* ----------------------------------------- Hermite Coulomb integrals R_{tuv} */
/* R[t][u][v] = R^0_{tuv}(alpha, X, Y, Z) for t+u+v <= L. */
typedef struct { double v[LTOT + 1][LTOT + 1][LTOT + 1]; } rtab_t;

static void hermite_R(int L, double alpha, double X, double Y, double Zc, rtab_t *out) {
  static __thread double Rn[LTOT + 1][LTOT + 1][LTOT + 1][LTOT + 1];
  double F[LTOT + 1];
  or_boys(L, alpha * (X * X + Y * Y + Zc * Zc), F);
  double f = 1.0;
  for (int n = 0; n <= L; ++n) { Rn[n][0][0][0] = f * F[n]; f *= -2.0 * alpha; }
  for (int n = L - 1; n >= 0; --n) {
    for (int s = 1; s <= L - n; ++s)
      for (int t = 0; t <= s; ++t)
        for (int u = 0; u <= s - t; ++u) {
          int v = s - t - u;
          double r;
          if (t > 0) {
            r = X * Rn[n + 1][t - 1][u][v];
            if (t > 1) r += (t - 1) * Rn[n + 1][t - 2][u][v];
          } else if (u > 0) {
            r = Y * Rn[n + 1][t][u - 1][v];
            if (u > 1) r += (u - 1) * Rn[n + 1][t][u - 2][v];
          } else {
            r = Zc * Rn[n + 1][t][u][v - 1];
            if (v > 1) r += (v - 1) * Rn[n + 1][t][u][v - 2];
          }
          Rn[n][t][u][v] = r;
        }
  }
  for (int t = 0; t <= L; ++t)
    for (int u = 0; u <= L - t; ++u)
      for (int v = 0; v <= L - t - u; ++v) out->v[t][u][v] = Rn[0][t][u][v];
}

/* ---------------------------------------------- primitive pair E tables */
typedef struct {
  double p, P[3];
  double E[3][NE][NE][NT];
} pairE_t;

static void pair_setup(double a, const double *A, double b, const double *B,
                       int imax, int jmax, pairE_t *pe) {
  pe->p = a + b;
  for (int d = 0; d < 3; ++d) {
    pe->P[d] = (a * A[d] + b * B[d]) / pe->p;
    hermite_E(imax, jmax, a, b, A[d] - B[d], pe->E[d]);
  }
}

/* primitive overlap <a|b> for Cartesian exponent tuples */
static double prim_S(const pairE_t *pe, const int *ia, const int *ib) {
  if (ia[0] < 0 || ia[1] < 0 || ia[2] < 0 || ib[0] < 0 || ib[1] < 0 || ib[2] < 0) return 0.0;
  return pe->E[0][ia[0]][ib[0]][0] * pe->E[1][ia[1]][ib[1]][0] * pe->E[2][ia[2]][ib[2]][0] *
         pow(M_PI / pe->p, 1.5);
}

/* primitive kinetic -1/2 <a|lap|b>; b is the exponent of the ket */
static double prim_T(const pairE_t *pe, const int *ia, const int *ib, double b) {
  double t = 0.0;
  for (int d = 0; d < 3; ++d) {
    int jp[3] = {ib[0], ib[1], ib[2]}, jm[3] = {ib[0], ib[1], ib[2]};
    jp[d] += 2; jm[d] -= 2;
    int j = ib[d];
    t += 4.0 * b * b * prim_S(pe, ia, jp) - 2.0 * b * (2 * j + 1) * prim_S(pe, ia, ib) +
         j * (j - 1) * prim_S(pe, ia, jm);
  }
  return -0.5 * t;
}

/* primitive <a| 1/|r-C| |b> (positive), and its derivative with respect to C_dir */
static double prim_V(const pairE_t *pe, const int *ia, const int *ib, const double *C,
                     int dir /* -1: value, 0..2: d/dC_dir */) {
  if (ia[0] < 0 || ia[1] < 0 || ia[2] < 0 || ib[0] < 0 || ib[1] < 0 || ib[2] < 0) return 0.0;
  static __thread rtab_t R;
  int L = ia[0] + ia[1] + ia[2] + ib[0] + ib[1] + ib[2] + (dir >= 0 ? 1 : 0);
  hermite_R(L, pe->p, pe->P[0] - C[0], pe->P[1] - C[1], pe->P[2] - C[2], &R);
  double s = 0.0;
  for (int t = 0; t <= ia[0] + ib[0]; ++t)
    for (int u = 0; u <= ia[1] + ib[1]; ++u)
      for (int v = 0; v <= ia[2] + ib[2]; ++v) {
        double e = pe->E[0][ia[0]][ib[0]][t] * pe->E[1][ia[1]][ib[1]][u] *
                   pe->E[2][ia[2]][ib[2]][v];
        double r;
        if (dir < 0) r = R.v[t][u][v];
        else if (dir == 0) r = -R.v[t + 1][u][v];
        else if (dir == 1) r = -R.v[t][u + 1][v];
        else r = -R.v[t][u][v + 1];
        s += e * r;
      }
  return 2.0 * M_PI / pe->p * s;
}

/* ------------------------------------------------ one-electron matrices */
/* S, T, V (V includes -Z_C for every nucleus); n x n row-major. */
void or_one_electron(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                     const int *pofs, const int *bf, const double *exps, const double *coefs,
                     int natom, const double *xyz, const int *Z, double *S, double *T,
                     double *V) {
  memset(S, 0, sizeof(double) * nbf * nbf);
  memset(T, 0, sizeof(double) * nbf * nbf);
  memset(V, 0, sizeof(double) * nbf * nbf);
  for (int a = 0; a < nsh; ++a)
    for (int b = 0; b < nsh; ++b) {
      const double *A = xyz + 3 * atom[a], *B = xyz + 3 * atom[b];
      for (int ka = 0; ka < nprim[a]; ++ka)
        for (int kb = 0; kb < nprim[b]; ++kb) {
          double al = exps[pofs[a] + ka], be = exps[pofs[b] + kb];
          double cc = coefs[pofs[a] + ka] * coefs[pofs[b] + kb];
          pairE_t pe;
          pair_setup(al, A, be, B, l[a] + 1, l[b] + 3, &pe);
          for (int i = 0; i < ncart(l[a]); ++i)
            for (int j = 0; j < ncart(l[b]); ++j) {
              int ia[3], ib[3];
              cart(l[a], i, &ia[0], &ia[1], &ia[2]);
              cart(l[b], j, &ib[0], &ib[1], &ib[2]);
              double f = cc * comp_norm(ia[0], ia[1], ia[2]) * comp_norm(ib[0], ib[1], ib[2]);
              int mu = bf[a] + i, nu = bf[b] + j;
              S[mu * nbf + nu] += f * prim_S(&pe, ia, ib);
              T[mu * nbf + nu] += f * prim_T(&pe, ia, ib, be);
              double v = 0.0;
              for (int c = 0; c < natom; ++c) v -= Z[c] * prim_V(&pe, ia, ib, xyz + 3 * c, -1);
              V[mu * nbf + nu] += f * v;
            }
        }
    }
}

/* ------------------------------------------------------------- ERIs */
/* Primitive (ab|cd) for Cartesian tuples from the two pair tables. */
static double prim_eri(const pairE_t *ab, const pairE_t *cd, const rtab_t *R, const int *ia,
                       const int *ib, const int *ic, const int *id) {
  for (int d = 0; d < 3; ++d)
    if (ia[d] < 0 || ib[d] < 0 || ic[d] < 0 || id[d] < 0) return 0.0;
  double s = 0.0;
  for (int t = 0; t <= ia[0] + ib[0]; ++t)
    for (int u = 0; u <= ia[1] + ib[1]; ++u)
      for (int v = 0; v <= ia[2] + ib[2]; ++v) {
        double e1 = ab->E[0][ia[0]][ib[0]][t] * ab->E[1][ia[1]][ib[1]][u] *
                    ab->E[2][ia[2]][ib[2]][v];
        if (e1 == 0.0) continue;
        double inner = 0.0;
        for (int tau = 0; tau <= ic[0] + id[0]; ++tau)
          for (int nu = 0; nu <= ic[1] + id[1]; ++nu)
            for (int phi = 0; phi <= ic[2] + id[2]; ++phi) {
              double e2 = cd->E[0][ic[0]][id[0]][tau] * cd->E[1][ic[1]][id[1]][nu] *
                          cd->E[2][ic[2]][id[2]][phi];
              double sg = ((tau + nu + phi) & 1) ? -1.0 : 1.0;
              inner += sg * e2 * R->v[t + tau][u + nu][v + phi];
            }
        s += e1 * inner;
      }
  double p = ab->p, q = cd->p;
  return 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * s;
}

/* Contracted shell-quartet block out[i][j][k][l] (function indices within
 * shells a,b,c,d).  With deriv != NULL, also fills the 12 centre-derivative
 * blocks deriv[centre*3+dir][...] (centre 0..3 = a,b,c,d). */
static void shell_quartet(const basis_t *bs, int a, int b, int c, int d, double *out,
                          double *deriv) {
  int sh[4] = {a, b, c, d}, L[4], nc[4];
  const double *X[4];
  for (int k = 0; k < 4; ++k) {
    L[k] = bs->l[sh[k]];
    nc[k] = ncart(L[k]);
    X[k] = bs->xyz + 3 * bs->atom[sh[k]];
  }
  int nblk = nc[0] * nc[1] * nc[2] * nc[3];
  if (out) memset(out, 0, sizeof(double) * nblk);
  if (deriv) memset(deriv, 0, sizeof(double) * 12 * nblk);
  int raise = deriv ? 1 : 0;
  int Ltot = L[0] + L[1] + L[2] + L[3] + raise;
  static __thread pairE_t pab, pcd;
  static __thread rtab_t R;
  /* tuple tables per function */
  int tup[4][ncart(LMAX)][3];
  double cn[4][ncart(LMAX)];
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < nc[k]; ++i) {
      cart(L[k], i, &tup[k][i][0], &tup[k][i][1], &tup[k][i][2]);
      cn[k][i] = comp_norm(tup[k][i][0], tup[k][i][1], tup[k][i][2]);
    }
  for (int ka = 0; ka < bs->nprim[a]; ++ka)
    for (int kb = 0; kb < bs->nprim[b]; ++kb) {
      double al = bs->exps[bs->pofs[a] + ka], be = bs->exps[bs->pofs[b] + kb];
      double cab = bs->coefs[bs->pofs[a] + ka] * bs->coefs[bs->pofs[b] + kb];
      pair_setup(al, X[0], be, X[1], L[0] + raise, L[1] + raise, &pab);
      for (int kc = 0; kc < bs->nprim[c]; ++kc)
        for (int kd = 0; kd < bs->nprim[d]; ++kd) {
          double ga = bs->exps[bs->pofs[c] + kc], de = bs->exps[bs->pofs[d] + kd];
          double ccd = bs->coefs[bs->pofs[c] + kc] * bs->coefs[bs->pofs[d] + kd];
          pair_setup(ga, X[2], de, X[3], L[2] + raise, L[3] + raise, &pcd);
          double p = pab.p, q = pcd.p, alpha = p * q / (p + q);
          hermite_R(Ltot, alpha, pab.P[0] - pcd.P[0], pab.P[1] - pcd.P[1],
                    pab.P[2] - pcd.P[2], &R);
          double ex[4] = {al, be, ga, de};
          double w = cab * ccd;
          int n = 0;
          for (int i = 0; i < nc[0]; ++i)
            for (int j = 0; j < nc[1]; ++j)
              for (int k = 0; k < nc[2]; ++k)
                for (int m = 0; m < nc[3]; ++m, ++n) {
                  const int *t4[4] = {tup[0][i], tup[1][j], tup[2][k], tup[3][m]};
                  double f = w * cn[0][i] * cn[1][j] * cn[2][k] * cn[3][m];
                  if (out) out[n] += f * prim_eri(&pab, &pcd, &R, t4[0], t4[1], t4[2], t4[3]);
                  if (!deriv) continue;
                  for (int cen = 0; cen < 4; ++cen)
                    for (int dir = 0; dir < 3; ++dir) {
                      int up[3] = {t4[cen][0], t4[cen][1], t4[cen][2]};
                      int dn[3] = {t4[cen][0], t4[cen][1], t4[cen][2]};
                      up[dir] += 1; dn[dir] -= 1;
                      const int *u4[4] = {t4[0], t4[1], t4[2], t4[3]};
                      const int *d4[4] = {t4[0], t4[1], t4[2], t4[3]};
                      u4[cen] = up; d4[cen] = dn;
                      double v = 2.0 * ex[cen] * prim_eri(&pab, &pcd, &R, u4[0], u4[1], u4[2], u4[3]);
                      if (t4[cen][dir] > 0)
                        v -= t4[cen][dir] * prim_eri(&pab, &pcd, &R, d4[0], d4[1], d4[2], d4[3]);
                      deriv[(cen * 3 + dir) * nblk + n] += f * v;
                    }
                }
        }
    }
}

/* Public: contracted block for one shell quartet (for tests). */
void or_eri_quartet(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                    const int *pofs, const int *bf, const double *exps, const double *coefs,
                    const double *xyz, int a, int b, int c, int d, double *out,
                    double *deriv) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  shell_quartet(&bs, a, b, c, d, out, deriv);
}

/* Full n^4 ERI tensor (tiny bases only), every shell quartet computed directly. */
void or_eri_tensor(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                   const int *pofs, const int *bf, const double *exps, const double *coefs,
                   const double *xyz, double *out) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  size_t n = nbf;
  double blk[6 * 6 * 6 * 6 * 4];
  for (int a = 0; a < nsh; ++a)
    for (int b = 0; b < nsh; ++b)
      for (int c = 0; c < nsh; ++c)
        for (int d = 0; d < nsh; ++d) {
          shell_quartet(&bs, a, b, c, d, blk, NULL);
          int na = ncart(l[a]), nb = ncart(l[b]), nc = ncart(l[c]), nd = ncart(l[d]), q = 0;
          for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j)
              for (int k = 0; k < nc; ++k)
                for (int m = 0; m < nd; ++m, ++q)
                  out[(((bf[a] + i) * n + bf[b] + j) * n + bf[c] + k) * n + bf[d] + m] = blk[q];
        }
}

/* Q[a*nsh+b] = sqrt(max over functions of |(mn|mn)|) */
void or_schwarz(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                const int *pofs, const int *bf, const double *exps, const double *coefs,
                const double *xyz, double *Q) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < nsh; ++a) {
    double blk[6 * 6 * 6 * 6];
    for (int b = 0; b <= a; ++b) {
      shell_quartet(&bs, a, b, a, b, blk, NULL);
      int na = ncart(l[a]), nb = ncart(l[b]);
      double m = 0.0;
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          double v = fabs(blk[((i * nb + j) * na + i) * nb + j]);
          if (v > m) m = v;
        }
      Q[a * nsh + b] = Q[b * nsh + a] = sqrt(m);
    }
  }
}

/* Canonical quartet list: a>=b, c>=d, pair(ab) >= pair(cd), Q_ab Q_cd >= tau. */
static int canonical_list(int nsh, const double *Q, double tau, int **list_out) {
  int npair = nsh * (nsh + 1) / 2;
  int *pa = malloc(sizeof(int) * npair), *pb = malloc(sizeof(int) * npair);
  for (int a = 0, k = 0; a < nsh; ++a)
    for (int b = 0; b <= a; ++b, ++k) { pa[k] = a; pb[k] = b; }
  size_t cap = 1024, n = 0;
  int *lst = malloc(sizeof(int) * 4 * cap);
  for (int i = 0; i < npair; ++i)
    for (int j = 0; j <= i; ++j) {
      int a = pa[i], b = pb[i], c = pa[j], d = pb[j];
      if (tau > 0.0 && Q[a * nsh + b] * Q[c * nsh + d] < tau) continue;
      if (n == cap) { cap *= 2; lst = realloc(lst, sizeof(int) * 4 * cap); }
      lst[4 * n] = a; lst[4 * n + 1] = b; lst[4 * n + 2] = c; lst[4 * n + 3] = d;
      ++n;
    }
  free(pa); free(pb);
  *list_out = lst;
  return (int)n;
}

/* The 8 index permutations (ij|kl) of a shell quartet, as position maps. */
static const int PERM8[8][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
                                {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};

/* Distinct shell permutations of (a,b,c,d); returns count, fills which[]. */
static int distinct_perms(const int *s, int *which) {
  int n = 0;
  for (int p = 0; p < 8; ++p) {
    int t[4] = {s[PERM8[p][0]], s[PERM8[p][1]], s[PERM8[p][2]], s[PERM8[p][3]]}, dup = 0;
    for (int q = 0; q < n && !dup; ++q) {
      int u[4] = {s[PERM8[which[q]][0]], s[PERM8[which[q]][1]], s[PERM8[which[q]][2]],
                  s[PERM8[which[q]][3]]};
      dup = (t[0] == u[0] && t[1] == u[1] && t[2] == u[2] && t[3] == u[3]);
    }
    if (!dup) which[n++] = p;
  }
  return n;
}

/* Direct J and K for density P (n x n), Schwarz threshold tau (<=0: none).
 * Returns the number of shell quartets evaluated. */
long or_jk(int nsh, int nbf, const int *l, const int *atom, const int *nprim, const int *pofs,
           const int *bf, const double *exps, const double *coefs, const double *xyz,
           const double *Q, double tau, const double *P, double *J, double *K) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  int *lst;
  int nq = canonical_list(nsh, Q, tau, &lst);
  size_t n = nbf;
  memset(J, 0, sizeof(double) * n * n);
  memset(K, 0, sizeof(double) * n * n);
#pragma omp parallel
  {
    double *Jt = calloc(n * n, sizeof(double)), *Kt = calloc(n * n, sizeof(double));
    double blk[6 * 6 * 6 * 6];
#pragma omp for schedule(dynamic, 16)
    for (int q = 0; q < nq; ++q) {
      int s[4] = {lst[4 * q], lst[4 * q + 1], lst[4 * q + 2], lst[4 * q + 3]};
      shell_quartet(&bs, s[0], s[1], s[2], s[3], blk, NULL);
      int nc4[4], b0[4];
      for (int k = 0; k < 4; ++k) { nc4[k] = ncart(l[s[k]]); b0[k] = bf[s[k]]; }
      int which[8], np = distinct_perms(s, which);
      int e = 0;
      for (int i = 0; i < nc4[0]; ++i)
        for (int j = 0; j < nc4[1]; ++j)
          for (int k = 0; k < nc4[2]; ++k)
            for (int m = 0; m < nc4[3]; ++m, ++e) {
              int g[4] = {b0[0] + i, b0[1] + j, b0[2] + k, b0[3] + m};
              double v = blk[e];
              for (int pp = 0; pp < np; ++pp) {
                const int *pm = PERM8[which[pp]];
                int mu = g[pm[0]], nu = g[pm[1]], la = g[pm[2]], si = g[pm[3]];
                Jt[mu * n + nu] += v * P[la * n + si];
                Kt[mu * n + la] += v * P[nu * n + si];
              }
            }
    }
#pragma omp critical
    for (size_t i = 0; i < n * n; ++i) { J[i] += Jt[i]; K[i] += Kt[i]; }
    free(Jt); free(Kt);
  }
  free(lst);
  return nq;
}

/* Timing sample of or_jk: the same digestion over every stride-th quartet of
 * the canonical screened list only, on nthreads threads (<= 0: the OpenMP
 * default).  J and K receive that partial sum.  Returns the number of shell
 * quartets evaluated. */
long or_jk_sample(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                  const int *pofs, const int *bf, const double *exps, const double *coefs,
                  const double *xyz, const double *Q, double tau, const double *P, int stride,
                  int nthreads, double *J, double *K) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  int *lst;
  int nq = canonical_list(nsh, Q, tau, &lst);
  if (stride < 1) stride = 1;
  int ns = (nq + stride - 1) / stride;
  for (int q = 0; q < ns; ++q)
    for (int k = 0; k < 4; ++k) lst[4 * q + k] = lst[4 * (q * stride) + k];
  size_t n = nbf;
  memset(J, 0, sizeof(double) * n * n);
  memset(K, 0, sizeof(double) * n * n);
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  int nt = 1;
  (void)nthreads;
#endif
#pragma omp parallel num_threads(nt)
  {
    double *Jt = calloc(n * n, sizeof(double)), *Kt = calloc(n * n, sizeof(double));
    double blk[6 * 6 * 6 * 6];
#pragma omp for schedule(dynamic, 16)
    for (int q = 0; q < ns; ++q) {
      int s4[4] = {lst[4 * q], lst[4 * q + 1], lst[4 * q + 2], lst[4 * q + 3]};
      shell_quartet(&bs, s4[0], s4[1], s4[2], s4[3], blk, NULL);
      int nc4[4], b0[4];
      for (int k = 0; k < 4; ++k) { nc4[k] = ncart(l[s4[k]]); b0[k] = bf[s4[k]]; }
      int which[8], np = distinct_perms(s4, which);
      int e = 0;
      for (int i = 0; i < nc4[0]; ++i)
        for (int j = 0; j < nc4[1]; ++j)
          for (int k = 0; k < nc4[2]; ++k)
            for (int m = 0; m < nc4[3]; ++m, ++e) {
              int g[4] = {b0[0] + i, b0[1] + j, b0[2] + k, b0[3] + m};
              double v = blk[e];
              for (int pp = 0; pp < np; ++pp) {
                const int *pm = PERM8[which[pp]];
                int mu = g[pm[0]], nu = g[pm[1]], la = g[pm[2]], si = g[pm[3]];
                Jt[mu * n + nu] += v * P[la * n + si];
                Kt[mu * n + la] += v * P[nu * n + si];
              }
            }
    }
#pragma omp critical
    for (size_t i = 0; i < n * n; ++i) { J[i] += Jt[i]; K[i] += Kt[i]; }
    free(Jt); free(Kt);
  }
  free(lst);
  return ns;
}

/* Two-electron gradient: g[atom][3] += 1/2 sum (mn|ls)^x [P_mn P_ls - kx/2 P_ml P_ns]
 * over all ordered index quartets, with the same Schwarz rule as or_jk; kx is
 * the share of exact exchange (1 for Hartree-Fock, 0.2 in B3LYP).
 * With amask != NULL only the atoms with amask[atom] != 0 are accumulated
 * (the others stay 0), and quartets with no shell on such an atom are skipped. */
static long grad_2e(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                    const int *pofs, const int *bf, const double *exps, const double *coefs,
                    const double *xyz, int natom, const double *Q, double tau, const double *P,
                    double kx, const int *amask, double *g) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  int *lst;
  int nq = canonical_list(nsh, Q, tau, &lst);
  if (amask) { /* keep the quartets that touch a selected atom */
    int m = 0;
    for (int q = 0; q < nq; ++q) {
      int hit = 0;
      for (int k = 0; k < 4; ++k) hit |= amask[atom[lst[4 * q + k]]] != 0;
      if (hit) {
        for (int k = 0; k < 4; ++k) lst[4 * m + k] = lst[4 * q + k];
        ++m;
      }
    }
    nq = m;
  }
  size_t n = nbf;
  memset(g, 0, sizeof(double) * 3 * natom);
#pragma omp parallel
  {
    double *gt = calloc(3 * natom, sizeof(double));
    double *der = malloc(sizeof(double) * 12 * 6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic, 8)
    for (int q = 0; q < nq; ++q) {
      int s[4] = {lst[4 * q], lst[4 * q + 1], lst[4 * q + 2], lst[4 * q + 3]};
      shell_quartet(&bs, s[0], s[1], s[2], s[3], NULL, der);
      int nc4[4], b0[4], at[4];
      for (int k = 0; k < 4; ++k) {
        nc4[k] = ncart(l[s[k]]); b0[k] = bf[s[k]]; at[k] = atom[s[k]];
      }
      int nblk = nc4[0] * nc4[1] * nc4[2] * nc4[3];
      int which[8], np = distinct_perms(s, which);
      int e = 0;
      for (int i = 0; i < nc4[0]; ++i)
        for (int j = 0; j < nc4[1]; ++j)
          for (int k = 0; k < nc4[2]; ++k)
            for (int m = 0; m < nc4[3]; ++m, ++e) {
              int gi[4] = {b0[0] + i, b0[1] + j, b0[2] + k, b0[3] + m};
              double gam = 0.0; /* sum over distinct permutations of the density factor */
              for (int pp = 0; pp < np; ++pp) {
                const int *pm = PERM8[which[pp]];
                int mu = gi[pm[0]], nu = gi[pm[1]], la = gi[pm[2]], si = gi[pm[3]];
                gam += 0.5 * (P[mu * n + nu] * P[la * n + si] - 0.5 * kx * P[mu * n + la] * P[nu * n + si]);
              }
              /* every permutation has the same centre derivatives (same centres) */
              for (int cen = 0; cen < 4; ++cen) {
                if (amask && !amask[at[cen]]) continue;
                for (int dir = 0; dir < 3; ++dir)
                  gt[3 * at[cen] + dir] += gam * der[(cen * 3 + dir) * nblk + e];
              }
            }
    }
#pragma omp critical
    for (int i = 0; i < 3 * natom; ++i) g[i] += gt[i];
    free(gt); free(der);
  }
  free(lst);
  return nq;
}

long or_grad_2e(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                const int *pofs, const int *bf, const double *exps, const double *coefs,
                const double *xyz, int natom, const double *Q, double tau, const double *P,
                double *g) {
  return grad_2e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, natom, Q, tau, P, 1.0, NULL, g);
}

long or_grad_2e_kx(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                   const int *pofs, const int *bf, const double *exps, const double *coefs,
                   const double *xyz, int natom, const double *Q, double tau, const double *P,
                   double kx, double *g) {
  return grad_2e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, natom, Q, tau, P, kx, NULL, g);
}

long or_grad_2e_atoms(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                      const int *pofs, const int *bf, const double *exps, const double *coefs,
                      const double *xyz, int natom, const double *Q, double tau, const double *P,
                      const int *amask, double *g) {
  return grad_2e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz, natom, Q, tau, P, 1.0, amask, g);
}

/* One-electron gradient: g[atom][3] = sum P_mn dH_mn/dX - sum W_mn dS_mn/dX,
 * with the Hellmann-Feynman operator term of every nucleus.  With amask !=
 * NULL only the atoms with amask[atom] != 0 are accumulated (the others stay
 * 0): the bra and ket terms of the shells on them and their operator terms. */
static void grad_1e(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                    const int *pofs, const int *bf, const double *exps, const double *coefs,
                    int natom, const double *xyz, const int *Z, const double *P, const double *W,
                    const int *amask, double *g) {
  size_t n = nbf;
  memset(g, 0, sizeof(double) * 3 * natom);
#pragma omp parallel
  {
  double *gt = calloc(3 * natom, sizeof(double));
#pragma omp for schedule(dynamic)
  for (int a = 0; a < nsh; ++a)
    for (int b = 0; b < nsh; ++b) {
      const int bra_on = !amask || amask[atom[a]], ket_on = !amask || amask[atom[b]];
      const double *A = xyz + 3 * atom[a], *B = xyz + 3 * atom[b];
      for (int ka = 0; ka < nprim[a]; ++ka)
        for (int kb = 0; kb < nprim[b]; ++kb) {
          double al = exps[pofs[a] + ka], be = exps[pofs[b] + kb];
          double cc = coefs[pofs[a] + ka] * coefs[pofs[b] + kb];
          pairE_t pe;
          pair_setup(al, A, be, B, l[a] + 1, l[b] + 4, &pe);
          for (int i = 0; i < ncart(l[a]); ++i)
            for (int j = 0; j < ncart(l[b]); ++j) {
              int ia[3], ib[3];
              cart(l[a], i, &ia[0], &ia[1], &ia[2]);
              cart(l[b], j, &ib[0], &ib[1], &ib[2]);
              double f = cc * comp_norm(ia[0], ia[1], ia[2]) * comp_norm(ib[0], ib[1], ib[2]);
              int mu = bf[a] + i, nu = bf[b] + j;
              double pmn = P[mu * n + nu], wmn = W[mu * n + nu];
              for (int dir = 0; dir < 3; ++dir) {
                /* derivative with respect to the bra centre (atom of shell a) */
                if (bra_on) {
                int up[3] = {ia[0], ia[1], ia[2]}, dn[3] = {ia[0], ia[1], ia[2]};
                up[dir] += 1; dn[dir] -= 1;
                double dS = 2 * al * prim_S(&pe, up, ib) - ia[dir] * prim_S(&pe, dn, ib);
                double dT = 2 * al * prim_T(&pe, up, ib, be) - ia[dir] * prim_T(&pe, dn, ib, be);
                double dV = 0.0;
                for (int c = 0; c < natom; ++c) {
                  double v = 2 * al * prim_V(&pe, up, ib, xyz + 3 * c, -1);
                  if (ia[dir] > 0) v -= ia[dir] * prim_V(&pe, dn, ib, xyz + 3 * c, -1);
                  dV -= Z[c] * v;
                }
                gt[3 * atom[a] + dir] += f * (pmn * (dT + dV) - wmn * dS);
                }
                /* derivative with respect to the ket centre (atom of shell b) */
                if (ket_on) {
                int up2[3] = {ib[0], ib[1], ib[2]}, dn2[3] = {ib[0], ib[1], ib[2]};
                up2[dir] += 1; dn2[dir] -= 1;
                double dS = 2 * be * prim_S(&pe, ia, up2) - ib[dir] * prim_S(&pe, ia, dn2);
                double dT = 2 * be * prim_T(&pe, ia, up2, be) - ib[dir] * prim_T(&pe, ia, dn2, be);
                double dV = 0.0;
                for (int c = 0; c < natom; ++c) {
                  double v = 2 * be * prim_V(&pe, ia, up2, xyz + 3 * c, -1);
                  if (ib[dir] > 0) v -= ib[dir] * prim_V(&pe, ia, dn2, xyz + 3 * c, -1);
                  dV -= Z[c] * v;
                }
                gt[3 * atom[b] + dir] += f * (pmn * (dT + dV) - wmn * dS);
                }
                /* operator centre of every nucleus c */
                for (int c = 0; c < natom; ++c)
                  if (!amask || amask[c])
                    gt[3 * c + dir] += f * pmn * (-Z[c]) * prim_V(&pe, ia, ib, xyz + 3 * c, dir);
              }
            }
        }
    }
#pragma omp critical
  for (int i = 0; i < 3 * natom; ++i) g[i] += gt[i];
  free(gt);
  }
}

void or_grad_1e(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                const int *pofs, const int *bf, const double *exps, const double *coefs,
                int natom, const double *xyz, const int *Z, const double *P, const double *W,
                double *g) {
  grad_1e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, natom, xyz, Z, P, W, NULL, g);
}

void or_grad_1e_atoms(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                      const int *pofs, const int *bf, const double *exps, const double *coefs,
                      int natom, const double *xyz, const int *Z, const double *P,
                      const double *W, const int *amask, double *g) {
  grad_1e(nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, natom, xyz, Z, P, W, amask, g);
}

/* J and K blocks of selected shell pairs, by direct summation over every
 * ordered ket shell pair (no permutational symmetry):
 *   J_mn = sum_{c,d} sum_{l in c, s in d} (mn|ls) P_ls,  included when
 *          Q_ab Q_cd >= tau,
 *   K_mn = sum_{c,d} sum_{l in c, s in d} (ml|ns) P_ls,  included when
 *          Q_ac Q_bd >= tau,
 * for m in shell pa[i], n in shell pb[i]; the same Schwarz rule as or_jk
 * (the rule of the canonical quartet each term belongs to).  Only the
 * elements of the selected blocks of J and K (n x n) are written. */
void or_jk_pairs(int nsh, int nbf, const int *l, const int *atom, const int *nprim,
                 const int *pofs, const int *bf, const double *exps, const double *coefs,
                 const double *xyz, const double *Q, double tau, const double *P, int npairs,
                 const int *pa, const int *pb, double *J, double *K) {
  basis_t bs = {nsh, nbf, l, atom, nprim, pofs, bf, exps, coefs, xyz};
  size_t n = nbf;
  for (int i = 0; i < npairs; ++i) {
    const int a = pa[i], b = pb[i], na = ncart(l[a]), nb = ncart(l[b]);
    double Jb[36] = {0}, Kb[36] = {0};
#pragma omp parallel
    {
      double Jt[36] = {0}, Kt[36] = {0};
      double blk[6 * 6 * 6 * 6];
#pragma omp for schedule(dynamic)
      for (int c = 0; c < nsh; ++c)
        for (int d = 0; d < nsh; ++d) {
          const int nc = ncart(l[c]), nd = ncart(l[d]);
          if (tau <= 0.0 || Q[a * nsh + b] * Q[c * nsh + d] >= tau) {
            shell_quartet(&bs, a, b, c, d, blk, NULL);
            for (int u = 0; u < na; ++u)
              for (int v = 0; v < nb; ++v)
                for (int x = 0; x < nc; ++x)
                  for (int y = 0; y < nd; ++y)
                    Jt[u * nb + v] += blk[((u * nb + v) * nc + x) * nd + y] *
                                      P[(bf[c] + x) * n + bf[d] + y];
          }
          if (tau <= 0.0 || Q[a * nsh + c] * Q[b * nsh + d] >= tau) {
            shell_quartet(&bs, a, c, b, d, blk, NULL);
            for (int u = 0; u < na; ++u)
              for (int x = 0; x < nc; ++x)
                for (int v = 0; v < nb; ++v)
                  for (int y = 0; y < nd; ++y)
                    Kt[u * nb + v] += blk[((u * nc + x) * nb + v) * nd + y] *
                                      P[(bf[c] + x) * n + bf[d] + y];
          }
        }
#pragma omp critical
      for (int k = 0; k < na * nb; ++k) { Jb[k] += Jt[k]; Kb[k] += Kt[k]; }
    }
    for (int u = 0; u < na; ++u)
      for (int v = 0; v < nb; ++v) {
        J[(bf[a] + u) * n + bf[b] + v] = Jb[u * nb + v];
        K[(bf[a] + u) * n + bf[b] + v] = Kb[u * nb + v];
      }
  }
}
