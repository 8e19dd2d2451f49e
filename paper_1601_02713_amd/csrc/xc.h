// Exchange-correlation quadrature for closed-shell B3LYP, the paper's level of
// theory (Section 3.1: B3LYP/6-31G*): a density functional integrated on a
// molecular grid replaces 80% of the exact exchange.
//
// Grid: per atom, kXcRad radial points of Becke's mapping r = R (1+x)/(1-x)
// of Gauss-Chebyshev nodes of the second kind (R = 1.0 bohr for H, 0.6 bohr
// otherwise) times a product angular grid of kXcTheta Gauss-Legendre nodes in
// cos(theta) and 2 kXcTheta equally spaced phi; Becke's fuzzy-cell weights
// (three iterations of p(mu) = 1.5 mu - 0.5 mu^3, no size adjustment).
// Functional (Stephens et al. 1994): 0.8 Slater + 0.72 Becke-88 gradient
// correction + 0.19 VWN (RPA fit) + 0.81 LYP, with 0.2 of the exact exchange;
// closed shell, rho the total density and sigma = |grad rho|^2.
//
// Per run of consecutive instances with equal basis size and per chunk of G
// grid points: basis values B, function-major [inst][n][G] (xc_basis);
// Z = B P (a strided-batched GEMM); per point the density, its gradient (basis
// gradients recomputed on the fly, never stored) and the functional, and
// X = w (v_rho B / 2 + 2 v_sigma grad rho . grad B) written over Z
// (xc_point); then V = X^T B accumulated over the chunks (a batched GEMM
// per slice of the chunk's points and their sum) and V + V^T at the end.
#pragma once
#include "common.h"

namespace bscf {

constexpr int kXcRad = 60;
constexpr int kXcTheta = 12;
constexpr int kXcAng = 2 * kXcTheta * kXcTheta;     // angular points per radial shell
constexpr int kXcPerAtom = kXcRad * kXcAng;
constexpr double kXcA0 = 0.20;                      // exact-exchange share
constexpr double kXcRhoMin = 1e-14;                 // smaller densities contribute nothing

struct XcGridArgs {
  int npts;                 // points of this instance (atoms x kXcPerAtom)
  int natoms;
  const double* xyz;        // [natoms][3] of the instance
  const double* Z;          // [natoms]
  const double* rad_r;      // [2][kXcRad]: H, then others
  const double* rad_w;
  const double* ang_u;      // [kXcAng][3]
  const double* ang_w;      // [kXcAng]
  double* pts;              // [npts][4]: x, y, z, weight (Becke weight included)
  const double* inv_sep;    // [natoms][natoms] 1/|R_A - R_B| (weight gradient only)
};

struct XcChunkArgs {
  int G;                    // chunk width: the leading dimension of B and Z
  int g0;                   // first point of the chunk (per instance)
  int n;                    // basis functions of every instance of the run
  int first;                // first instance of the run
  const int* npts;          // [ninst] grid points per instance
  const long long* pt_off;  // [ninst] first point of each instance in pts
  const int* sh_off;        // [ninst] first shell of each instance
  const int* nsh;           // [ninst] shells per instance
  const Shell* shells;
  const double* sh_exp;
  const double* sh_coef;
  const double* pts;        // [sum npts][4]: x, y, z, weight
  double* B;                // [count][n][G] basis values
  double* Z;                // [count][n][G]: B P, then (xc_point) X
  double* part;             // [count][G / 256] partial sums of w e per block
};

// Sparse form (instances of one group with the same atoms, e.g. beads): the
// grid is cut into chunks of kXcSparseShells radial shells of one atom times
// one of kXcSectors angular sectors (cos(theta) >= 0 or < 0 times
// sin(phi) >= 0 or < 0: 6 x 12 of the 12 x 24 product nodes), and a chunk
// takes only the basis shells whose values (or gradients) can exceed
// kXcShellEps somewhere on it (a distance bound, union over the group's
// instances), numbered compactly: B, Z [count][ns][G], P and V through the
// compact-to-local function map.  The sparse kernels run blocks of kXcSB
// threads (G is a multiple of it).
constexpr int kXcSparseShells = 8;
constexpr int kXcSectors = 4;
constexpr int kXcSectorAng = kXcAng / kXcSectors;               // 72
constexpr int kXcSparseG = kXcSparseShells * kXcSectorAng;      // 576 points, 9 x 64
constexpr int kXcSB = 64;
constexpr double kXcShellEps = 1e-14;

// One launch covers nch chunks of a bucket (chunks of similar size, padded to
// W compact functions) times the count instances of a run: slot z =
// chunk * count + instance.  Per chunk (chunk metadata, kXcMeta ints): first
// point of its radial block (atom * kXcPerAtom + first shell * kXcAng),
// points, first entry and length of its shell list, first entry and length of
// its function map, sector.  Point g of a chunk is radial row g / kXcSectorAng
// of the block at angular node sec_ang[sector][g % kXcSectorAng].
struct XcSparseArgs {
  int G;                    // points per chunk slot (multiple of kXcSB)
  int W;                    // padded compact functions per slot
  int nch, count;           // chunks and instances of the launch
  int first;                // first instance of the run
  int n;                    // basis functions per instance
  const int* meta;          // [nch][kXcMeta]: p0, gcnt, sh0, nsh, f0, ns, sector
  const int* sec_ang;       // [kXcSectors][kXcSectorAng] angular nodes of each sector
  const int* sh_list;       // shells (local to the instance) of all chunks
  const int* sh_cbf;        // first compact function of each listed shell
  const int* fmap;          // local function of each compact one, all chunks
  const int* sh_off;        // per instance: first global shell
  const Shell* shells;
  const double* sh_exp;
  const double* sh_coef;
  const long long* pt_off;  // per instance: first grid point
  const double* pts;
  const long long* moff;    // per instance: matrix offset
  const double* P;
  double* B;                // [slot][W][G]
  double* Z;                // [slot][W][G]: B Ps, then X
  double* Ps;               // [slot][W][W] compact density (column-major, zero padded)
  double* Vs;               // [slot][W][W] X^T B
  double* V;                // V_xc (column-major per instance, + V^T at the end)
  double* part;             // [slot][G / kXcSB] partial sums of w e
};
constexpr int kXcMeta = 7;

// max_nsh: the longest shell list of the launch's chunks
void launch_xc_sparse_basis(const XcSparseArgs& a, int max_nsh, hipStream_t s);
void launch_xc_sparse_gather(const XcSparseArgs& a, hipStream_t s);
void launch_xc_sparse_point(const XcSparseArgs& a, hipStream_t s);
// V += Vs through the function maps (atomics: chunks of one instance overlap)
void launch_xc_sparse_scatter(const XcSparseArgs& a, hipStream_t s);
// exc[first + i] += the partial sums of instance i over the launch's chunks, in order
void launch_xc_sparse_reduce(const XcSparseArgs& a, double* exc, hipStream_t s);

// Nuclear gradient of E_xc at fixed density (closed shell, sparse form).  Per
// point of a chunk of atom B, for every atom A != B (point held fixed):
//   d(w e)/dR_A = w_rad w_ang e dW_B/dR_A
//                 + w [v_rho drho/dR_A + v_sigma dsigma/dR_A],
//   drho/dR_A   = -2 sum_{m on A} grad phi_m Z_m,
//   dsigma/dR_A = -4 sum_{m on A} [(H_m grad rho) Z_m + grad phi_m Y_m],
// Z_m = sum_n P_mn phi_n, Y_m = sum_n P_mn (grad rho . grad phi_n), H_m the
// Hessian of phi_m, W_B the Becke weight; atom B takes minus the sum over
// A != B (each point's term is unchanged by a rigid translation, the point
// moving with its atom).
//
// xc_sparse_gpoint: per point rho, grad rho and the functional; writes
// D_m = grad rho . grad phi_m over B (the compact functions), the factors
// gf[slot][5][G] = {w v_rho, w v_sigma, grad rho} and e per grid point into
// eg (zero where rho is below kXcRhoMin).  Then Y = D Ps (a batched GEMM).
void launch_xc_sparse_gpoint(const XcSparseArgs& a, double* gf, double* eg, hipStream_t s);
// xc_sparse_force: the basis-function term, one thread per (point, shell),
// summed per block and shell into grad[3 * atom] (dE/dR) with atomics
void launch_xc_sparse_force(const XcSparseArgs& a, int max_nsh, const double* gf,
                            const double* Y, const int* atom_off, double* grad, hipStream_t s);
// xc_weight_grad: the Becke-weight term of one instance's points (the grid
// arguments of the instance; eg its energy densities; grad its atoms' rows)
void launch_xc_weight_grad(const XcGridArgs& a, const double* eg, double* grad, hipStream_t s);

void launch_xc_grid(const XcGridArgs& a, hipStream_t s);
// count instances of the run, at most max_nsh shells each
void launch_xc_basis(const XcChunkArgs& a, int count, int max_nsh, hipStream_t s);
void launch_xc_point(const XcChunkArgs& a, int count, hipStream_t s);
// exc[first + i] += sum of the G / 256 partial sums of instance i, in order
void launch_xc_reduce(const XcChunkArgs& a, int count, double* exc, hipStream_t s);
// V[i] = (add ? V[i] : 0) + sum over s < S of Vp[i][s] (n x n each), i < count
void launch_xc_slice_sum(int n, int count, int S, const double* Vp, double* V, bool add,
                         hipStream_t s);
// count n x n matrices (stride n^2): M <- M + M^T
void launch_xc_symmetrize(int n, int count, double* V, hipStream_t s);
// e, v_rho, v_sigma of the closed-shell B3LYP energy density at n points
void launch_xc_functional(int n, const double* rho, const double* sigma, double* e, double* vr,
                          double* vs, hipStream_t s);

}  // namespace bscf
