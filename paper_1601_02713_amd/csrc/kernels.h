// Argument blocks and host launchers of the non-class kernels.
#pragma once
#include "common.h"

namespace bscf {

struct PrimPairSetupArgs {
  int nprim;
  const int* prim_pair_owner;  // shell-pair index of each primitive pair
  const ShellPair* pairs;
  const Shell* shells;
  const double* sh_exp;        // per shell primitive: exponent
  const double* sh_coef;       // per shell primitive: normalised contraction coefficient
  PrimPair* prims;
};

struct OneEArgs {
  int ntasks;                  // shell pairs a >= b of this class (one block each)
  const int* task_a;
  const int* task_b;
  const Shell* shells;
  const double* sh_exp;
  const double* sh_coef;
  const int* natoms;
  const int* atom_off;
  const double* atom_xyz;
  const double* atom_Z;
  const int* nbf;
  const long long* moff;
  const double* boys64;
  double* S;
  double* T;
  double* V;
};

struct Grad1EArgs {
  int ntasks;                  // shell pairs a >= b of this class (one block each)
  const int* task_a;
  const int* task_b;
  const Shell* shells;
  const double* sh_exp;
  const double* sh_coef;
  const int* natoms;
  const int* atom_off;
  const double* atom_xyz;
  const double* atom_Z;
  const int* nbf;
  const long long* moff;
  const double* boys64;
  const double* P;
  const double* W;
  const int* active;
  double* grad;                // [total atoms][3]
};

void launch_prim_pairs(const PrimPairSetupArgs& a, hipStream_t s);
void launch_onee(int la, int lb, const OneEArgs& a, hipStream_t s);
// The work rows of one quartet class for launch_row_keep: keep (may be NULL)
// receives per row the kets that pass; cq, cpq (and c32, may be NULL) receive
// per instance the kept quartets, primitive quartets (and kept quartets past
// each row's FP64 prefix, row.pad).  block0 is set by the launcher.
struct RowKeepClass {
  const WorkRow* rows;
  int nrows;
  int block0;
  int* keep;
  double* cq;
  double* cpq;
  double* c32;
};
constexpr int kRowKeepMaxClasses = 24;
struct RowKeepSet {
  int nclass;
  RowKeepClass cls[kRowKeepMaxClasses];
};
// keep[r] = kets of work row r with Q_ab Q_cd min(dpmax[inst], 1) >= tau for
// the rows of active instances, with the counts added to cq, cpq (c32), for
// ncls classes in one launch per kRowKeepMaxClasses (jk.hip)
void launch_row_keep(const RowKeepClass* cls, int ncls, const int* kets, const ShellPair* pairs,
                     const Shell* shells, const double* Q, const double* dpmax, const int* active,
                     double tau, int ninst, hipStream_t s);
void launch_grad1e(int la, int lb, const Grad1EArgs& a, hipStream_t s);

// ---- ket-list-position buffers of the Fock build (jk.hip) ----
// Position pos of the ket list holds shell pair kets[pos] = (c, d); its
// component e = k * ncart(l_d) + l is stored at [e * nk_total + pos], so the
// lanes of a wavefront that take consecutive positions touch consecutive
// doubles.
struct KetPosArgs {
  int nk_total;
  const int* kets;
  const ShellPair* pairs;
  const Shell* shells;
  const long long* moff;
  const int* nbf;
};
// dst[t] = src[map[t]] for the n primitive-pair records of the ket order
void launch_gather_prims(int n, const int* map, const PrimPair* src, PrimPair* dst, hipStream_t s);
// Pk[e * nk_total + pos] = P(c_k, d_l)
// Pm[pm_off[i] + s nsh[i] + t] = max |P| over the block of local shells s, t
// of instance i (density-weighted screening of the gradient)
void launch_shell_pmax(int ninst, int max_nsh, const int* shell_off, const int* nsh,
                       const long long* pm_off, const Shell* shells, const long long* moff,
                       const int* nbf, const double* P, double* Pm, hipStream_t s);
void launch_gather_pk(const KetPosArgs& a, int max_ncd, const double* P, double* Pk,
                      hipStream_t s);
// J(c_k, d_l) += Jk[e * nk_total + pos], then Jk = 0 (ready for the next build)
void launch_jk_finalize(const KetPosArgs& a, int max_ncd, double* Jk, double* J, hipStream_t s);
// Deterministic builds: the fold in the fixed-point words of fx_add (common.h),
// the conversion of n fixed-point values to FP64 and a clear of n words.
void launch_jk_finalize_fx(const KetPosArgs& a, int max_ncd, unsigned long long* Jk,
                           unsigned long long* J, hipStream_t s);
void launch_fx_to_double(long long n, const unsigned long long* fx, double* out, hipStream_t s);
void launch_fill_u64(long long n, unsigned long long* p, hipStream_t s);

// ---- dense per-instance helpers (scf.hip) ----
struct BatchInfo {
  int ninst;
  const int* nbf;
  const long long* moff;
  const int* active;
};

void launch_fill(double* p, long long n, double v, hipStream_t s);
// F = H + (J + J^T)/2 - kx (K + K^T)/4 (+ Vxc); E[i] = Tr[P(H+F')]/2 + Exc[i] +
// Enuc[i] with F' = F without Vxc (Hartree-Fock: kx = 1, no Vxc, Exc);
// instances masked out by b.active (when non-NULL) keep their F and E
void launch_fock_assemble(const BatchInfo& b, int max_n, const double* H, const double* J,
                          const double* K, const double* P, const double* Enuc, double* F,
                          double* E, hipStream_t s, double kx = 1.0, const double* Vxc = nullptr,
                          const double* Exc = nullptr);
// out = A - A^T per instance; the largest |out| of every 32 x 32 tile goes to
// the scratch after the first ninst entries of emax (room for
// ninst * ceil(max_n/32)^2 doubles), reduced into emax[i] by launch_convergence
void launch_antisym(const BatchInfo& b, int max_n, const double* A, double* out, double* emax,
                    hipStream_t s);
// DIIS: store F, e in slot; update B row; solve; Fbar = sum c F
struct DiisArgs {
  int ninst;
  int max_vec;
  const int* nbf;
  const long long* moff;
  const int* active;
  long long stride;      // per-slot stride of the history buffers (total matrix size)
  double* Fhist;         // [max_vec][mtot]
  double* Ehist;
  double* B;             // [ninst][max_vec][max_vec]
  int* count;            // per instance number of stored vectors
  int* head;             // per instance next slot
  double* coef;          // [ninst][max_vec]
};
void launch_diis_store(const DiisArgs& d, int max_n, const double* F, const double* e,
                       hipStream_t s);
void launch_diis_extrapolate(const DiisArgs& d, int max_n, double* Fbar, hipStream_t s);
// convergence flags of the active instances: emax[i] = max |A - A^T| from
// launch_antisym's tile maxima; niter[i] += 1; instance i converges (leaves
// the active set) when it has a previous energy and |E - Eprev| < etol and
// emax < ctol.  No host value changes between iterations, so the launch can
// be replayed from a graph.
void launch_convergence(int ninst, int max_n, const int* nbf, const double* E, double* Eprev,
                        double* emax, double etol, double ctol, int* active, int* niter,
                        int* status, hipStream_t s);
// SP2 purification (scf.hip).  launch_sp2_bounds: Gershgorin intervals of
// the rows of each instance's F' (bounds[inst][row] = (lo, hi), room for
// ninst * max_n pairs).  launch_sp2_init: X = (hi I - (F' + F'^T)/2)/(hi - lo)
// over their union, and conv[inst] = -1.  launch_sp2_step (step k): Xn = X^2
// or 2X - X^2, as the trace rule on st_in (the statistics of X) decides; X and
// Xn must not overlap.  Both store, per 32 x 32 tile of the result, its
// (Tr, Tr^2) partial at st[(inst * sp2_tiles(max_n) + tile) * 2]; the sum over
// an instance's tiles is its (Tr X, Tr X^2).  conv_out[inst] = the first step
// j <= k whose X_j met Tr X - Tr X^2 < idem_tol and |Tr X - nocc| < trace_tol
// (-1 if none), given conv_in from step k - 1 (from init for k = 0); an
// instance with j + 2 <= k is finished and Xn = X.  conv_in and conv_out must
// be distinct arrays of ninst ints.  Instances masked out by b.active are
// skipped.
void launch_sp2_bounds(const BatchInfo& b, int max_n, const double* F, double* bounds,
                       hipStream_t s);
void launch_sp2_init(const BatchInfo& b, int max_n, const double* F, const double* bounds,
                     double* X, double* st, int* conv, hipStream_t s);
void launch_sp2_step(const BatchInfo& b, int max_n, const int* nocc, const double* X, double* Xn,
                     const double* st_in, double* st_out, int step, double idem_tol,
                     double trace_tol, const int* conv_in, int* conv_out, hipStream_t s);
int sp2_tiles(int max_n);
// dP = P - Pprev and dpmax[i] = max |dP| of instance i (the instances of b);
// dpmax needs room for ninst + ninst * ceil(max_n/32)^2 doubles (scf.hip)
void launch_density_change(const BatchInfo& b, int max_n, const double* P, const double* Pprev,
                           double* dP, double* dpmax, hipStream_t s);
// out[0, na) = a and out[na, na + nb) = b (int arrays; one copy to the host
// then reads both)
void launch_concat_ints(const int* a, int na, const int* b, int nb, int* out, hipStream_t s);
// P_new -> P for active instances
void launch_commit(const BatchInfo& b, int max_n, const double* Pnew, double* P, hipStream_t s);
// nuclear repulsion energy and gradient per instance
void launch_nuclear(int ninst, const int* natoms, const int* atom_off, const double* xyz,
                    const double* Z, double* Enuc, double* grad, int want_grad, hipStream_t s);
// dst = alpha * src (or its transpose) per instance (all instances if active is NULL)
void launch_scale_copy(const BatchInfo& b, int max_n, const double* src, double* dst,
                       double alpha, int transpose, hipStream_t s);

// out[i*(m_max+1)+m] = F_m(T[i]) by the device Boys function (FP64 or FP32 body)
void launch_boys_eval(int m_max, int n, const double* T, double* out, int fp32,
                      const double* tab64, const float* tab32, hipStream_t s);

// Boys table on the host (Gauss-Legendre quadrature of the defining integral)
void boys_table_host(double* tab /* kBoysRows * kBoysCols */);

}  // namespace bscf
