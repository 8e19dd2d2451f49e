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
// Per instance and chunk of grid points: basis values and gradients B, Bx,
// By, Bz, function-major [n][points] (xc_basis), Z = B P (a GEMM), density,
// gradient and the functional per point with
// X = w (v_rho B / 2 + 2 v_sigma grad rho . grad B) written over Z (xc_point),
// then V += X^T B (a GEMM); V_xc = V + V^T at the end.
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
};

struct XcChunkArgs {
  int g0, ng;               // points [g0, g0 + ng) of the instance
  int n;                    // basis functions of the instance
  int sh0, nsh;             // its shells in the shell table
  const Shell* shells;
  const double* sh_exp;
  const double* sh_coef;
  const double* pts;        // the instance's [npts][4]
  double* B;                // [n][ng] (function-major) values
  double* Bx;               // and gradients
  double* By;
  double* Bz;
  double* Z;                // [n][ng]: B P, then (xc_point) X
  double* exc;              // accumulates sum_g w e
};

void launch_xc_grid(const XcGridArgs& a, hipStream_t s);
void launch_xc_basis(const XcChunkArgs& a, hipStream_t s);
void launch_xc_point(const XcChunkArgs& a, hipStream_t s);
// V (n x n, row-major) = M + M^T, in place
void launch_xc_symmetrize(int n, double* V, hipStream_t s);
// e, v_rho, v_sigma of the closed-shell B3LYP energy density at n points
void launch_xc_functional(int n, const double* rho, const double* sigma, double* e, double* vr,
                          double* vs, hipStream_t s);

}  // namespace bscf
