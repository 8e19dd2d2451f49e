// Exchange-correlation quadrature kernels (see xc.h).  Basis values and the
// GEMM operands are function-major, [n][points], so consecutive threads of a
// point-parallel kernel touch consecutive addresses.
#include "xc.h"

#include <algorithm>
#include <cmath>

namespace bscf {
namespace {

// ---------------------------------------------------------------- functional

struct Xc {
  double e, vr, vs;
};

__device__ __forceinline__ Xc b3lyp(double rho, double sigma) {
  const double t = cbrt(1.0 / rho);             // rho^(-1/3)
  const double r13 = 1.0 / t;                   // rho^(1/3)
  // Slater exchange, 0.8
  const double cx = 0.75 * cbrt(3.0 / M_PI);
  double e = -0.8 * cx * rho * r13;
  double vr = -0.8 * (4.0 / 3.0) * cx * r13;
  double vs = 0.0;
  // Becke 88 gradient correction, 0.72: per spin rho_s = rho/2,
  // x = |grad rho_s| / rho_s^(4/3), e = -2 beta rho_s^(4/3) g(x),
  // g = x^2 / (1 + 6 beta x asinh x)
  {
    const double beta = 0.0042;
    const double rs = 0.5 * rho;
    const double rs13 = cbrt(rs), rs43 = rs * rs13;
    const double x2 = 0.25 * sigma / (rs43 * rs43);
    const double x = sqrt(x2);
    const double ash = asinh(x);
    const double den = 1.0 + 6.0 * beta * x * ash;
    const double g = x2 / den;
    // g'(x) / x, finite at x = 0
    const double gpx = (2.0 * den - x * (6.0 * beta * ash + 6.0 * beta * x / sqrt(1.0 + x2))) / (den * den);
    e += 0.72 * (-2.0 * beta * rs43 * g);
    vr += 0.72 * (-(4.0 / 3.0) * beta * rs13 * (g - x2 * gpx));
    // dx/dsigma = x / (2 sigma) and x^2 / sigma = 1 / (4 rho_s^(8/3))
    vs += 0.72 * (-beta * rs43 * gpx * 0.25 / (rs43 * rs43));
  }
  // VWN correlation (RPA fit), 0.19: e = rho eps(rs), v = eps - rs/3 deps/drs
  {
    const double A = 0.0310907, x0 = -0.409286, b = 13.0720, c = 42.7198;
    const double rsv = cbrt(3.0 / (4.0 * M_PI * rho));
    const double x = sqrt(rsv);
    const double X = x * x + b * x + c, X0 = x0 * x0 + b * x0 + c;
    const double Q = sqrt(4.0 * c - b * b);
    const double at = atan(Q / (2.0 * x + b));
    const double eps = A * (log(x * x / X) + 2.0 * b / Q * at -
                            b * x0 / X0 * (log((x - x0) * (x - x0) / X) + 2.0 * (b + 2.0 * x0) / Q * at));
    const double q2 = (2.0 * x + b) * (2.0 * x + b) + Q * Q;
    const double deps_dx = A * (2.0 / x - (2.0 * x + b) / X - 4.0 * b / q2 -
                                b * x0 / X0 * (2.0 / (x - x0) - (2.0 * x + b) / X - 4.0 * (b + 2.0 * x0) / q2));
    const double deps_drs = deps_dx / (2.0 * x);
    e += 0.19 * rho * eps;
    vr += 0.19 * (eps - rsv / 3.0 * deps_drs);
  }
  // LYP correlation, 0.81 (closed shell):
  // e = -a rho/(1 + d t) - a b g(rho) h(rho, sigma), t = rho^(-1/3),
  // g = exp(-c t)/(1 + d t), h = C_F rho - rho^(-5/3) sigma (1/24 + 7 delta/72),
  // delta = c t + d t/(1 + d t)
  {
    const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
    const double cf = 0.3 * cbrt(3.0 * M_PI * M_PI) * cbrt(3.0 * M_PI * M_PI);
    const double dt1 = 1.0 + d * t;
    const double delta = c * t + d * t / dt1;
    const double g = exp(-c * t) / dt1;
    const double r53 = t * t * t * t * t;         // rho^(-5/3)
    const double h = cf * rho - r53 * sigma * (1.0 / 24.0 + 7.0 * delta / 72.0);
    const double dt_drho = -t / (3.0 * rho);
    const double ddelta = (c + d / (dt1 * dt1)) * dt_drho;
    const double dg = g * delta / (3.0 * rho);
    const double dh = cf - sigma * (-(5.0 / 3.0) * r53 / rho * (1.0 / 24.0 + 7.0 * delta / 72.0) +
                                    r53 * (7.0 / 72.0) * ddelta);
    const double d1 = -a * (1.0 / dt1 + (d * t / 3.0) / (dt1 * dt1));
    e += 0.81 * (-a * rho / dt1 - a * b * g * h);
    vr += 0.81 * (d1 - a * b * (dg * h + g * dh));
    vs += 0.81 * (a * b * g * r53 * (1.0 / 24.0 + 7.0 * delta / 72.0));
  }
  return {e, vr, vs};
}

// ------------------------------------------------------------------- kernels

__global__ void xc_grid_kernel(XcGridArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npts) return;
  const int A = p / kXcPerAtom, k = p - A * kXcPerAtom;
  const int i = k / kXcAng, j = k - i * kXcAng;
  const int tab = a.Z[A] == 1.0 ? 0 : 1;
  const double r = a.rad_r[tab * kXcRad + i];
  const double x = a.xyz[3 * A] + r * a.ang_u[3 * j];
  const double y = a.xyz[3 * A + 1] + r * a.ang_u[3 * j + 1];
  const double z = a.xyz[3 * A + 2] + r * a.ang_u[3 * j + 2];
  // Becke cell function of every atom at the point; the owner's share
  double own = 0.0, tot = 0.0;
  for (int B = 0; B < a.natoms; ++B) {
    const double dxB = x - a.xyz[3 * B], dyB = y - a.xyz[3 * B + 1], dzB = z - a.xyz[3 * B + 2];
    const double rB = sqrt(dxB * dxB + dyB * dyB + dzB * dzB);
    double PB = 1.0;
    for (int C = 0; C < a.natoms && PB > 0.0; ++C) {
      if (C == B) continue;
      const double dxC = x - a.xyz[3 * C], dyC = y - a.xyz[3 * C + 1], dzC = z - a.xyz[3 * C + 2];
      const double rC = sqrt(dxC * dxC + dyC * dyC + dzC * dzC);
      const double ex = a.xyz[3 * B] - a.xyz[3 * C], ey = a.xyz[3 * B + 1] - a.xyz[3 * C + 1],
                   ez = a.xyz[3 * B + 2] - a.xyz[3 * C + 2];
      double mu = (rB - rC) / sqrt(ex * ex + ey * ey + ez * ez);
      for (int it = 0; it < 3; ++it) mu = 1.5 * mu - 0.5 * mu * mu * mu;
      PB *= 0.5 * (1.0 - mu);
    }
    tot += PB;
    if (B == A) own = PB;
  }
  const double w = a.rad_w[tab * kXcRad + i] * a.ang_w[j] * (tot > 0.0 ? own / tot : 0.0);
  double* o = a.pts + 4LL * p;
  o[0] = x;
  o[1] = y;
  o[2] = z;
  o[3] = w;
}

__device__ __forceinline__ double dfact(int n) {   // n!! for n in -1..3
  return n == 3 ? 3.0 : 1.0;
}

// one thread per (point, shell): values and gradients of the shell's
// Cartesian components (lexicographic), each normalised to unit self-overlap
__global__ __launch_bounds__(256) void xc_basis_kernel(XcChunkArgs a) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  if (gl >= a.ng) return;
  const Shell sh = a.shells[a.sh0 + blockIdx.y];
  const double* pt = a.pts + 4LL * (a.g0 + gl);
  const double dx = pt[0] - sh.x, dy = pt[1] - sh.y, dz = pt[2] - sh.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  double rad = 0.0, drad = 0.0;   // sum c e^{-a r^2} and its r^2-derivative
  for (int k = 0; k < sh.nprim; ++k) {
    const double al = a.sh_exp[sh.prim0 + k];
    const double e = a.sh_coef[sh.prim0 + k] * exp(-al * r2);
    rad += e;
    drad -= al * e;
  }
  const long long ng = a.ng;
  int f = sh.bf;
  const int l = sh.l;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly, ++f) {
      const int lz = l - lx - ly;
      const double cn = rsqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
      const double px = lx == 0 ? 1.0 : (lx == 1 ? dx : dx * dx);
      const double py = ly == 0 ? 1.0 : (ly == 1 ? dy : dy * dy);
      const double pz = lz == 0 ? 1.0 : (lz == 1 ? dz : dz * dz);
      const double qx = lx == 0 ? 0.0 : (lx == 1 ? 1.0 : 2.0 * dx);   // d/dx of x^lx
      const double qy = ly == 0 ? 0.0 : (ly == 1 ? 1.0 : 2.0 * dy);
      const double qz = lz == 0 ? 0.0 : (lz == 1 ? 1.0 : 2.0 * dz);
      const double ang = px * py * pz;
      const long long o = (long long)f * ng + gl;
      a.B[o] = cn * ang * rad;
      a.Bx[o] = cn * (qx * py * pz * rad + ang * 2.0 * dx * drad);
      a.By[o] = cn * (px * qy * pz * rad + ang * 2.0 * dy * drad);
      a.Bz[o] = cn * (px * py * qz * rad + ang * 2.0 * dz * drad);
    }
}

// one thread per point: rho = sum B Z, grad rho = 2 sum grad(B) Z, the
// functional, and X = w (v_rho B / 2 + 2 v_sigma grad rho . grad B) over Z
__global__ __launch_bounds__(256) void xc_point_kernel(XcChunkArgs a) {
  __shared__ double red[256];
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  double ew = 0.0;
  if (gl < a.ng) {
    const long long ng = a.ng;
    double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int m = 0; m < a.n; ++m) {
      const long long o = (long long)m * ng + gl;
      const double z = a.Z[o];
      rho += a.B[o] * z;
      gx += a.Bx[o] * z;
      gy += a.By[o] * z;
      gz += a.Bz[o] * z;
    }
    gx *= 2.0;
    gy *= 2.0;
    gz *= 2.0;
    const double w = a.pts[4LL * (a.g0 + gl) + 3];
    double cr = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    if (rho > kXcRhoMin) {
      const Xc f = b3lyp(rho, gx * gx + gy * gy + gz * gz);
      ew = w * f.e;
      cr = 0.5 * w * f.vr;
      cx = 2.0 * w * f.vs * gx;
      cy = 2.0 * w * f.vs * gy;
      cz = 2.0 * w * f.vs * gz;
    }
    for (int m = 0; m < a.n; ++m) {
      const long long o = (long long)m * ng + gl;
      a.Z[o] = cr * a.B[o] + cx * a.Bx[o] + cy * a.By[o] + cz * a.Bz[o];
    }
  }
  red[threadIdx.x] = ew;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0.0) atomicAdd(a.exc, red[0]);
}

__global__ void xc_symmetrize_kernel(int n, double* V) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || j < i) return;
  const double s = V[(long long)i * n + j] + V[(long long)j * n + i];
  V[(long long)i * n + j] = s;
  V[(long long)j * n + i] = s;
}

__global__ void xc_functional_kernel(int n, const double* rho, const double* sigma, double* e,
                                     double* vr, double* vs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const Xc f = b3lyp(rho[k], sigma[k]);
  e[k] = f.e;
  vr[k] = f.vr;
  vs[k] = f.vs;
}

}  // namespace

void launch_xc_grid(const XcGridArgs& a, hipStream_t s) {
  if (a.npts == 0) return;
  hipLaunchKernelGGL(xc_grid_kernel, dim3((a.npts + 255) / 256), dim3(256), 0, s, a);
}

void launch_xc_basis(const XcChunkArgs& a, hipStream_t s) {
  if (a.ng == 0 || a.nsh == 0) return;
  hipLaunchKernelGGL(xc_basis_kernel, dim3((a.ng + 255) / 256, a.nsh), dim3(256), 0, s, a);
}

void launch_xc_point(const XcChunkArgs& a, hipStream_t s) {
  if (a.ng == 0) return;
  hipLaunchKernelGGL(xc_point_kernel, dim3((a.ng + 255) / 256), dim3(256), 0, s, a);
}

void launch_xc_symmetrize(int n, double* V, hipStream_t s) {
  hipLaunchKernelGGL(xc_symmetrize_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, n, V);
}

void launch_xc_functional(int n, const double* rho, const double* sigma, double* e, double* vr,
                          double* vs, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(xc_functional_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, rho, sigma, e,
                     vr, vs);
}

}  // namespace bscf
