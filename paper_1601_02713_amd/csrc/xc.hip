// Exchange-correlation quadrature kernels (see xc.h).  Basis values and the
// GEMM operands are function-major, [inst][n][G], so consecutive threads of a
// point-parallel kernel touch consecutive addresses.  G is a multiple of 256.
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

// one thread per point (blocks of 64); dynamic LDS: the point's distance to
// every atom [natoms][64]
__global__ __launch_bounds__(64) void xc_grid_kernel(XcGridArgs a) {
  extern __shared__ double lds[];
  double* Rc = lds;   // [C][64]
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npts) return;
  const int A = p / kXcPerAtom, k = p - A * kXcPerAtom;
  const int i = k / kXcAng, j = k - i * kXcAng;
  const int tab = a.Z[A] == 1.0 ? 0 : 1;
  const double r = a.rad_r[tab * kXcRad + i];
  const double x = a.xyz[3 * A] + r * a.ang_u[3 * j];
  const double y = a.xyz[3 * A + 1] + r * a.ang_u[3 * j + 1];
  const double z = a.xyz[3 * A + 2] + r * a.ang_u[3 * j + 2];
  const int na = a.natoms;
  for (int C = 0; C < na; ++C) {
    const double dx = x - a.xyz[3 * C], dy = y - a.xyz[3 * C + 1], dz = z - a.xyz[3 * C + 2];
    Rc[C * 64 + threadIdx.x] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  // Becke cell function of every atom at the point; the owner's share
  double own = 0.0, tot = 0.0;
  for (int B = 0; B < na; ++B) {
    const double rB = Rc[B * 64 + threadIdx.x];
    double PB = 1.0;
    for (int C = 0; C < na && PB > 0.0; ++C) {
      if (C == B) continue;
      double mu = (rB - Rc[C * 64 + threadIdx.x]) * a.inv_sep[B * na + C];
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

// Values (and with Grad, gradients) of the Cartesian components of one shell
// at displacement (dx, dy, dz) from its centre, lexicographic order, each
// normalised to unit self-overlap: f(k, value, d/dx, d/dy, d/dz).
template <bool Grad, class Fn>
__device__ __forceinline__ void shell_eval(const Shell& sh, const double* __restrict__ ex,
                                           const double* __restrict__ co, double dx, double dy,
                                           double dz, Fn&& f) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  double rad = 0.0, drad = 0.0;   // sum c e^{-a r^2} and its r^2-derivative
  for (int k = 0; k < sh.nprim; ++k) {
    const double al = ex[sh.prim0 + k];
    const double e = co[sh.prim0 + k] * exp(-al * r2);
    rad += e;
    drad -= al * e;
  }
  const double gx = 2.0 * dx * drad, gy = 2.0 * dy * drad, gz = 2.0 * dz * drad;
  if (sh.l == 0) {
    f(0, rad, gx, gy, gz);
  } else if (sh.l == 1) {
    f(0, dx * rad, rad + dx * gx, dx * gy, dx * gz);
    f(1, dy * rad, dy * gx, rad + dy * gy, dy * gz);
    f(2, dz * rad, dz * gx, dz * gy, rad + dz * gz);
  } else {
    const double r3 = 0.57735026918962576451;   // 1/sqrt(3): xx, yy, zz
    f(0, r3 * dx * dx * rad, r3 * (2.0 * dx * rad + dx * dx * gx), r3 * dx * dx * gy,
      r3 * dx * dx * gz);
    f(1, dx * dy * rad, dy * rad + dx * dy * gx, dx * rad + dx * dy * gy, dx * dy * gz);
    f(2, dx * dz * rad, dz * rad + dx * dz * gx, dx * dz * gy, dx * rad + dx * dz * gz);
    f(3, r3 * dy * dy * rad, r3 * dy * dy * gx, r3 * (2.0 * dy * rad + dy * dy * gy),
      r3 * dy * dy * gz);
    f(4, dy * dz * rad, dy * dz * gx, dz * rad + dy * dz * gy, dy * rad + dy * dz * gz);
    f(5, r3 * dz * dz * rad, r3 * dz * dz * gx, r3 * dz * dz * gy,
      r3 * (2.0 * dz * rad + dz * dz * gz));
  }
}

// Values, gradients and Hessians (xx, xy, xz, yy, yz, zz) of the Cartesian
// components of one shell, same order and normalisation as shell_eval:
// f(k, v, g[3], h[6]).  Each component is s x^a y^b z^c R(r^2) with
// R = sum c e^{-alpha r^2}: d_i R = 2 x_i R', d_i d_j R = 2 delta_ij R' +
// 4 x_i x_j R''.
struct Mono {
  double v, d, dd;   // x^a and its first two derivatives
};
__device__ __forceinline__ Mono mono(int a, double x) {
  if (a == 0) return {1.0, 0.0, 0.0};
  if (a == 1) return {x, 1.0, 0.0};
  return {x * x, 2.0 * x, 2.0};
}
template <class Fn>
__device__ __forceinline__ void shell_eval_h(const Shell& sh, const double* __restrict__ ex,
                                             const double* __restrict__ co, double dx, double dy,
                                             double dz, Fn&& f) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  double R = 0.0, R1 = 0.0, R2 = 0.0;
  for (int k = 0; k < sh.nprim; ++k) {
    const double al = ex[sh.prim0 + k];
    const double e = co[sh.prim0 + k] * exp(-al * r2);
    R += e;
    R1 -= al * e;
    R2 += al * al * e;
  }
  const double d[3] = {dx, dy, dz};
  double Rg[3], Rh[6];
  {
    int q = 0;
    for (int i = 0; i < 3; ++i) {
      Rg[i] = 2.0 * d[i] * R1;
      for (int j = i; j < 3; ++j, ++q) Rh[q] = (i == j ? 2.0 * R1 : 0.0) + 4.0 * d[i] * d[j] * R2;
    }
  }
  auto comp = [&](int k, int a, int b, int c, double sc) {
    const Mono X = mono(a, dx), Y = mono(b, dy), Z = mono(c, dz);
    const double A = X.v * Y.v * Z.v;
    const double Ag[3] = {X.d * Y.v * Z.v, X.v * Y.d * Z.v, X.v * Y.v * Z.d};
    const double Ah[6] = {X.dd * Y.v * Z.v, X.d * Y.d * Z.v, X.d * Y.v * Z.d,
                          X.v * Y.dd * Z.v, X.v * Y.d * Z.d, X.v * Y.v * Z.dd};
    double g[3], h[6];
    int q = 0;
    for (int i = 0; i < 3; ++i) {
      g[i] = sc * (Ag[i] * R + A * Rg[i]);
      for (int j = i; j < 3; ++j, ++q)
        h[q] = sc * (Ah[q] * R + Ag[i] * Rg[j] + Ag[j] * Rg[i] + A * Rh[q]);
    }
    f(k, sc * A * R, g, h);
  };
  if (sh.l == 0) {
    comp(0, 0, 0, 0, 1.0);
  } else if (sh.l == 1) {
    comp(0, 1, 0, 0, 1.0);
    comp(1, 0, 1, 0, 1.0);
    comp(2, 0, 0, 1, 1.0);
  } else {
    const double r3 = 0.57735026918962576451;   // 1/sqrt(3): xx, yy, zz
    comp(0, 2, 0, 0, r3);
    comp(1, 1, 1, 0, 1.0);
    comp(2, 1, 0, 1, 1.0);
    comp(3, 0, 2, 0, r3);
    comp(4, 0, 1, 1, 1.0);
    comp(5, 0, 0, 2, r3);
  }
}

// one thread per (point, shell, instance of the run): the shell's basis
// values at the point (zero past the instance's last point)
__global__ __launch_bounds__(256) void xc_basis_kernel(XcChunkArgs a) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int zi = blockIdx.z, inst = a.first + zi;
  if ((int)blockIdx.y >= a.nsh[inst]) return;
  const Shell sh = a.shells[a.sh_off[inst] + blockIdx.y];
  double* Bc = a.B + ((size_t)zi * a.n + sh.bf) * a.G + gl;
  const int p = a.g0 + gl;
  const int nc = (sh.l + 1) * (sh.l + 2) / 2;
  if (p >= a.npts[inst]) {
    for (int k = 0; k < nc; ++k) Bc[(size_t)k * a.G] = 0.0;
    return;
  }
  const double* pt = a.pts + 4 * (a.pt_off[inst] + p);
  shell_eval<false>(sh, a.sh_exp, a.sh_coef, pt[0] - sh.x, pt[1] - sh.y, pt[2] - sh.z,
                    [&](int k, double v, double, double, double) { Bc[(size_t)k * a.G] = v; });
}

// one thread per point: rho = sum B Z, grad rho = 2 sum grad(B) Z (basis
// gradients recomputed), the functional, then
// X = w (v_rho B / 2 + 2 v_sigma grad rho . grad B) written over Z; each
// block's sum of w e to its partial-sum slot
__global__ __launch_bounds__(256) void xc_point_kernel(XcChunkArgs a) {
  __shared__ double red[256];
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int zi = blockIdx.y, inst = a.first + zi;
  const int p = a.g0 + gl;
  double ew = 0.0;
  if (p < a.npts[inst]) {
    const double* pt = a.pts + 4 * (a.pt_off[inst] + p);
    const double x = pt[0], y = pt[1], z = pt[2], w = pt[3];
    double* Zc = a.Z + (size_t)zi * a.n * a.G + gl;
    const Shell* sh0 = a.shells + a.sh_off[inst];
    const int nsh = a.nsh[inst];
    double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int s = 0; s < nsh; ++s) {
      const Shell sh = sh0[s];
      double* zf = Zc + (size_t)sh.bf * a.G;
      shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                       [&](int k, double v, double vx, double vy, double vz) {
                         const double zz = zf[(size_t)k * a.G];
                         rho += v * zz;
                         gx += vx * zz;
                         gy += vy * zz;
                         gz += vz * zz;
                       });
    }
    gx *= 2.0;
    gy *= 2.0;
    gz *= 2.0;
    double cr = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    if (rho > kXcRhoMin) {
      const Xc f = b3lyp(rho, gx * gx + gy * gy + gz * gz);
      ew = w * f.e;
      cr = 0.5 * w * f.vr;
      cx = 2.0 * w * f.vs * gx;
      cy = 2.0 * w * f.vs * gy;
      cz = 2.0 * w * f.vs * gz;
    }
    for (int s = 0; s < nsh; ++s) {
      const Shell sh = sh0[s];
      double* zf = Zc + (size_t)sh.bf * a.G;
      shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                       [&](int k, double v, double vx, double vy, double vz) {
                         zf[(size_t)k * a.G] = cr * v + cx * vx + cy * vy + cz * vz;
                       });
    }
  }
  red[threadIdx.x] = ew;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[(size_t)zi * (a.G / 256) + blockIdx.x] = red[0];
}

// one block per instance: its partial sums in a fixed order
__global__ __launch_bounds__(256) void xc_reduce_kernel(XcChunkArgs a, double* exc) {
  __shared__ double red[256];
  const int nb = a.G / 256;
  const double* pp = a.part + (size_t)blockIdx.x * nb;
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += pp[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) exc[a.first + blockIdx.x] += red[0];
}

// V[i] (+)= sum over s of Vp[i][s], s in order
__global__ void xc_slice_sum_kernel(int n, int S, const double* Vp, double* V, int add) {
  const size_t nn = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const double* src = Vp + (size_t)blockIdx.y * S * nn + e;
  double acc = add ? V[(size_t)blockIdx.y * nn + e] : 0.0;
  for (int s = 0; s < S; ++s) acc += src[(size_t)s * nn];
  V[(size_t)blockIdx.y * nn + e] = acc;
}

// ---------------------------------------------------------- sparse form

struct ChunkMeta {
  int p0, gcnt, sh0, nsh, f0, ns, sec;
};
__device__ __forceinline__ ChunkMeta chunk_meta(const int* m, int c) {
  const int* q = m + kXcMeta * c;
  return {q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
}
// grid point (within the instance) of point g of the chunk
__device__ __forceinline__ int chunk_point(const XcSparseArgs& a, const ChunkMeta& m, int g) {
  const int row = g / kXcSectorAng;
  return m.p0 + row * kXcAng + a.sec_ang[m.sec * kXcSectorAng + (g - row * kXcSectorAng)];
}

// grid (G / kXcSB, max_nsh + 1, slots): y < nsh a shell of the chunk, the
// last y the zero padding rows [ns, W)
__global__ __launch_bounds__(kXcSB) void xc_sparse_basis_kernel(XcSparseArgs a) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.z, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const ChunkMeta m = chunk_meta(a.meta, c);
  double* Bs = a.B + (size_t)slot * a.W * a.G + gl;
  if ((int)blockIdx.y == (int)gridDim.y - 1) {
    for (int k = m.ns; k < a.W; ++k) Bs[(size_t)k * a.G] = 0.0;
    return;
  }
  if ((int)blockIdx.y >= m.nsh) return;
  const int j = m.sh0 + blockIdx.y;
  const Shell sh = a.shells[a.sh_off[inst] + a.sh_list[j]];
  double* Bc = Bs + (size_t)a.sh_cbf[j] * a.G;
  const int nc = (sh.l + 1) * (sh.l + 2) / 2;
  if (gl >= m.gcnt) {
    for (int k = 0; k < nc; ++k) Bc[(size_t)k * a.G] = 0.0;
    return;
  }
  const double* pt = a.pts + 4 * (a.pt_off[inst] + chunk_point(a, m, gl));
  shell_eval<false>(sh, a.sh_exp, a.sh_coef, pt[0] - sh.x, pt[1] - sh.y, pt[2] - sh.z,
                    [&](int k, double v, double, double, double) { Bc[(size_t)k * a.G] = v; });
}

// Ps(i, j) = P(fmap[i], fmap[j]) inside the chunk's ns, zero in the padding
__global__ void xc_sparse_gather_kernel(XcSparseArgs a) {
  const int slot = blockIdx.y, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const long long ww = (long long)a.W * a.W;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ww) return;
  const ChunkMeta m = chunk_meta(a.meta, c);
  const int j = (int)(e / a.W), i = (int)(e - (long long)j * a.W);
  double v = 0.0;
  if (i < m.ns && j < m.ns)
    v = a.P[a.moff[inst] + (long long)a.fmap[m.f0 + i] * a.n + a.fmap[m.f0 + j]];
  a.Ps[slot * ww + e] = v;
}

// as xc_point_kernel over the chunk's shells
__global__ __launch_bounds__(kXcSB) void xc_sparse_point_kernel(XcSparseArgs a) {
  __shared__ double red[kXcSB];
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const ChunkMeta m = chunk_meta(a.meta, c);
  double ew = 0.0;
  if (gl < m.gcnt) {
    const double* pt = a.pts + 4 * (a.pt_off[inst] + chunk_point(a, m, gl));
    const double x = pt[0], y = pt[1], z = pt[2], w = pt[3];
    double* Zc = a.Z + (size_t)slot * a.W * a.G + gl;
    const Shell* sh0 = a.shells + a.sh_off[inst];
    double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j = m.sh0; j < m.sh0 + m.nsh; ++j) {
      const Shell sh = sh0[a.sh_list[j]];
      double* zf = Zc + (size_t)a.sh_cbf[j] * a.G;
      shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                       [&](int k, double v, double vx, double vy, double vz) {
                         const double zz = zf[(size_t)k * a.G];
                         rho += v * zz;
                         gx += vx * zz;
                         gy += vy * zz;
                         gz += vz * zz;
                       });
    }
    gx *= 2.0;
    gy *= 2.0;
    gz *= 2.0;
    double cr = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    if (rho > kXcRhoMin) {
      const Xc f = b3lyp(rho, gx * gx + gy * gy + gz * gz);
      ew = w * f.e;
      cr = 0.5 * w * f.vr;
      cx = 2.0 * w * f.vs * gx;
      cy = 2.0 * w * f.vs * gy;
      cz = 2.0 * w * f.vs * gz;
    }
    for (int j = m.sh0; j < m.sh0 + m.nsh; ++j) {
      const Shell sh = sh0[a.sh_list[j]];
      double* zf = Zc + (size_t)a.sh_cbf[j] * a.G;
      shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                       [&](int k, double v, double vx, double vy, double vz) {
                         zf[(size_t)k * a.G] = cr * v + cx * vx + cy * vy + cz * vz;
                       });
    }
  }
  red[threadIdx.x] = ew;
  __syncthreads();
  for (int st = kXcSB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[(size_t)slot * (a.G / kXcSB) + blockIdx.x] = red[0];
}

// V(fmap[i], fmap[j]) += Vs(i, j), column-major; the chunks of one instance
// add into the same matrix, so with atomics
__global__ void xc_sparse_scatter_kernel(XcSparseArgs a) {
  const int slot = blockIdx.y, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const long long ww = (long long)a.W * a.W;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ww) return;
  const ChunkMeta m = chunk_meta(a.meta, c);
  const int j = (int)(e / a.W), i = (int)(e - (long long)j * a.W);
  if (i >= m.ns || j >= m.ns) return;
  atomicAdd(&a.V[a.moff[inst] + (long long)a.fmap[m.f0 + j] * a.n + a.fmap[m.f0 + i]],
            a.Vs[slot * ww + e]);
}

// one block per instance: its partial sums over the launch's chunks, in order
__global__ __launch_bounds__(256) void xc_sparse_reduce_kernel(XcSparseArgs a, double* exc) {
  __shared__ double red[256];
  const int nb = a.G / kXcSB, zi = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < a.nch * nb; k += 256) {
    const int c = k / nb, b = k - c * nb;
    s += a.part[((size_t)c * a.count + zi) * nb + b];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) exc[a.first + zi] += red[0];
}

// ---------------------------------------------------------- gradient

// as xc_sparse_point_kernel up to the functional; then D over B, the point
// factors and the energy density (xc.h)
__global__ __launch_bounds__(kXcSB) void xc_sparse_gpoint_kernel(XcSparseArgs a, double* gf,
                                                               double* eg) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const ChunkMeta m = chunk_meta(a.meta, c);
  double* f = gf + (size_t)slot * 5 * a.G + gl;
  if (gl >= m.gcnt) {
    for (int k = 0; k < 5; ++k) f[(size_t)k * a.G] = 0.0;
    return;
  }
  const long long gp = a.pt_off[inst] + chunk_point(a, m, gl);
  const double* pt = a.pts + 4 * gp;
  const double x = pt[0], y = pt[1], z = pt[2], w = pt[3];
  const double* Zc = a.Z + (size_t)slot * a.W * a.G + gl;
  double* Dc = a.B + (size_t)slot * a.W * a.G + gl;
  const Shell* sh0 = a.shells + a.sh_off[inst];
  double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int j = m.sh0; j < m.sh0 + m.nsh; ++j) {
    const Shell sh = sh0[a.sh_list[j]];
    const double* zf = Zc + (size_t)a.sh_cbf[j] * a.G;
    shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                     [&](int k, double v, double vx, double vy, double vz) {
                       const double zz = zf[(size_t)k * a.G];
                       rho += v * zz;
                       gx += vx * zz;
                       gy += vy * zz;
                       gz += vz * zz;
                     });
  }
  gx *= 2.0;
  gy *= 2.0;
  gz *= 2.0;
  double cr = 0.0, cs = 0.0, e = 0.0;
  if (rho > kXcRhoMin) {
    const Xc fx = b3lyp(rho, gx * gx + gy * gy + gz * gz);
    cr = w * fx.vr;
    cs = w * fx.vs;
    e = fx.e;
  }
  f[0] = cr;
  f[(size_t)a.G] = cs;
  f[(size_t)2 * a.G] = gx;
  f[(size_t)3 * a.G] = gy;
  f[(size_t)4 * a.G] = gz;
  eg[gp] = e;
  for (int j = m.sh0; j < m.sh0 + m.nsh; ++j) {
    const Shell sh = sh0[a.sh_list[j]];
    double* df = Dc + (size_t)a.sh_cbf[j] * a.G;
    shell_eval<true>(sh, a.sh_exp, a.sh_coef, x - sh.x, y - sh.y, z - sh.z,
                     [&](int k, double, double vx, double vy, double vz) {
                       df[(size_t)k * a.G] = gx * vx + gy * vy + gz * vz;
                     });
  }
}

// grid (G / kXcSB, max_nsh, slots): y a shell of the chunk
__global__ __launch_bounds__(kXcSB) void xc_sparse_force_kernel(XcSparseArgs a, const double* gf,
                                                                const double* Y,
                                                                const int* atom_off,
                                                                double* grad) {
  __shared__ double red[3][kXcSB];
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.z, c = slot / a.count, zi = slot - c * a.count, inst = a.first + zi;
  const ChunkMeta m = chunk_meta(a.meta, c);
  if ((int)blockIdx.y >= m.nsh) return;   // the whole block
  const int j = m.sh0 + blockIdx.y;
  const Shell sh = a.shells[a.sh_off[inst] + a.sh_list[j]];
  const int own = atom_off[inst] + m.p0 / kXcPerAtom;   // the chunk's atom
  if (sh.atom == own) return;             // no net term (translation)
  double t[3] = {0.0, 0.0, 0.0};
  if (gl < m.gcnt) {
    const double* f = gf + (size_t)slot * 5 * a.G + gl;
    const double cr = f[0], cs = f[(size_t)a.G];
    if (cr != 0.0 || cs != 0.0) {
      const double g[3] = {f[(size_t)2 * a.G], f[(size_t)3 * a.G], f[(size_t)4 * a.G]};
      const double* pt = a.pts + 4 * (a.pt_off[inst] + chunk_point(a, m, gl));
      const size_t o = (size_t)slot * a.W * a.G + (size_t)a.sh_cbf[j] * a.G + gl;
      const double* zf = a.Z + o;
      const double* yf = Y + o;
      shell_eval_h(sh, a.sh_exp, a.sh_coef, pt[0] - sh.x, pt[1] - sh.y, pt[2] - sh.z,
                   [&](int k, double, const double* dv, const double* h) {
                     const double zz = zf[(size_t)k * a.G], yy = yf[(size_t)k * a.G];
                     const double hg[3] = {h[0] * g[0] + h[1] * g[1] + h[2] * g[2],
                                           h[1] * g[0] + h[3] * g[1] + h[4] * g[2],
                                           h[2] * g[0] + h[4] * g[1] + h[5] * g[2]};
                     for (int i = 0; i < 3; ++i)
                       t[i] += -2.0 * cr * dv[i] * zz - 4.0 * cs * (hg[i] * zz + dv[i] * yy);
                   });
    }
  }
  for (int i = 0; i < 3; ++i) red[i][threadIdx.x] = t[i];
  __syncthreads();
  for (int st = kXcSB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int i = 0; i < 3; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const double v = red[threadIdx.x][0];
    if (v != 0.0) {
      atomicAdd(&grad[3 * sh.atom + threadIdx.x], v);
      atomicAdd(&grad[3 * own + threadIdx.x], -v);
    }
  }
}

// Becke's s(mu) = (1 - p(p(p(mu)))) / 2 and s'/s (zero where s vanishes: mu
// = 1, where s' vanishes too)
__device__ __forceinline__ void becke_s(double mu, double& s, double& t) {
  const double p1 = 1.5 * mu - 0.5 * mu * mu * mu;
  const double p2 = 1.5 * p1 - 0.5 * p1 * p1 * p1;
  const double p3 = 1.5 * p2 - 0.5 * p2 * p2 * p2;
  s = 0.5 * (1.0 - p3);
  const double ds = -0.5 * 1.5 * (1.0 - p2 * p2) * 1.5 * (1.0 - p1 * p1) * 1.5 * (1.0 - mu * mu);
  t = s > 0.0 ? ds / s : 0.0;
}

// one thread per point of the instance (blocks of 64); dynamic LDS: the cell
// functions P_C and the distances r_C of the block's points [natoms][64] each
// and the block's gradient sums [natoms][3].  A cell function below kCellTiny is taken as zero here
// (its terms, bounded by it times |s'| <= 2.1, are far below rounding of the
// others), so per point only the pairs that touch a cell of the point do the
// work.
constexpr double kCellTiny = 1e-30;
__global__ __launch_bounds__(64) void xc_weight_grad_kernel(XcGridArgs a, const double* eg,
                                                            double* grad) {
  extern __shared__ double lds[];
  const int na = a.natoms;
  double* Pc = lds;              // [C][64]
  double* Rc = lds + 64 * na;    // [C][64]
  double* Gs = lds + 128 * na;   // [A][3]
  const double* iR = a.inv_sep;  // [C][D]
  for (int t = threadIdx.x; t < 3 * na; t += 64) Gs[t] = 0.0;
  __syncthreads();
  const int p = blockIdx.x * 64 + threadIdx.x;
  const double* R = a.xyz;
  double e = 0.0;
  if (p < a.npts) e = eg[p];
  if (e != 0.0) {
    const int B = p / kXcPerAtom, k = p - B * kXcPerAtom;
    const int i = k / kXcAng, jj = k - i * kXcAng;
    const int tab = a.Z[B] == 1.0 ? 0 : 1;
    const double r = a.rad_r[tab * kXcRad + i];
    const double x = R[3 * B] + r * a.ang_u[3 * jj];
    const double y = R[3 * B + 1] + r * a.ang_u[3 * jj + 1];
    const double z = R[3 * B + 2] + r * a.ang_u[3 * jj + 2];
    const double wra = a.rad_w[tab * kXcRad + i] * a.ang_w[jj];
    for (int C = 0; C < na; ++C) {
      const double dx = x - R[3 * C], dy = y - R[3 * C + 1], dz = z - R[3 * C + 2];
      Rc[C * 64 + threadIdx.x] = sqrt(dx * dx + dy * dy + dz * dz);
    }
    auto dist = [&](int C) { return Rc[C * 64 + threadIdx.x]; };
    double Zs = 0.0;
    for (int C = 0; C < na; ++C) {
      const double rC = dist(C);
      double PC = 1.0;
      for (int D = 0; D < na && PC >= kCellTiny; ++D) {
        if (D == C) continue;
        const double mu = (rC - dist(D)) * iR[C * na + D];
        const double p1 = 1.5 * mu - 0.5 * mu * mu * mu;
        const double p2 = 1.5 * p1 - 0.5 * p1 * p1 * p1;
        PC *= 0.5 * (1.0 - (1.5 * p2 - 0.5 * p2 * p2 * p2));
      }
      if (PC < kCellTiny) PC = 0.0;
      Pc[C * 64 + threadIdx.x] = PC;
      Zs += PC;
    }
    const double PB = Pc[B * 64 + threadIdx.x];
    if (Zs > 0.0 && PB > 0.0) {
      const double WB = PB / Zs, fac = wra * e / Zs;
      double gB[3] = {0.0, 0.0, 0.0};
      for (int A = 0; A < na; ++A) {
        if (A == B) continue;
        const double rA = dist(A), irA = 1.0 / rA;
        const double eA[3] = {(x - R[3 * A]) * irA, (y - R[3 * A + 1]) * irA,
                              (z - R[3 * A + 2]) * irA};
        // S = sum_{C != A} dP_C/dR_A, dPB = dP_B/dR_A, uA = dP_A/dR_A / P_A
        double S[3] = {0.0, 0.0, 0.0}, dPB[3] = {0.0, 0.0, 0.0}, uA[3] = {0.0, 0.0, 0.0};
        const double PA = Pc[A * 64 + threadIdx.x];
        for (int C = 0; C < na; ++C) {
          if (C == A) continue;
          const double PC = Pc[C * 64 + threadIdx.x];
          if (PC == 0.0 && PA == 0.0) continue;
          const double iRCA = iR[C * na + A], rC = dist(C);
          const double muCA = (rC - rA) * iRCA;
          const double dv[3] = {R[3 * C] - R[3 * A], R[3 * C + 1] - R[3 * A + 1],
                                R[3 * C + 2] - R[3 * A + 2]};
          if (PC != 0.0) {
            // dmu_CA/dR_A = e_A / R_CA + mu_CA (R_C - R_A) / R_CA^2
            double s, t;
            becke_s(muCA, s, t);
            for (int d = 0; d < 3; ++d) {
              const double v = PC * t * (eA[d] * iRCA + muCA * dv[d] * iRCA * iRCA);
              S[d] += v;
              if (C == B) dPB[d] = v;
            }
          }
          if (PA != 0.0) {
            // mu_AC = -mu_CA; dmu_AC/dR_A = -e_A / R_AC + mu_CA (R_A - R_C) / R_AC^2
            double s, t;
            becke_s(-muCA, s, t);
            for (int d = 0; d < 3; ++d) uA[d] += t * (-eA[d] * iRCA - muCA * dv[d] * iRCA * iRCA);
          }
        }
        for (int d = 0; d < 3; ++d) {
          const double v = fac * (dPB[d] - WB * (S[d] + PA * uA[d]));
          if (v != 0.0) atomicAdd(&Gs[3 * A + d], v);
          gB[d] -= v;
        }
      }
      for (int d = 0; d < 3; ++d) atomicAdd(&Gs[3 * B + d], gB[d]);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 3 * na; t += 64) {
    const double v = Gs[t];
    if (v != 0.0) atomicAdd(&grad[t], v);
  }
}

// M <- M + M^T for each of the run's n x n matrices
__global__ void xc_symmetrize_kernel(int n, double* V) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || j < i) return;
  double* M = V + (size_t)blockIdx.z * n * n;
  const double s = M[(size_t)i * n + j] + M[(size_t)j * n + i];
  M[(size_t)i * n + j] = s;
  M[(size_t)j * n + i] = s;
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
  hipLaunchKernelGGL(xc_grid_kernel, dim3((a.npts + 63) / 64), dim3(64),
                     sizeof(double) * 64 * (size_t)a.natoms, s, a);
}

void launch_xc_basis(const XcChunkArgs& a, int count, int max_nsh, hipStream_t s) {
  if (count == 0 || max_nsh == 0) return;
  hipLaunchKernelGGL(xc_basis_kernel, dim3(a.G / 256, max_nsh, count), dim3(256), 0, s, a);
}

void launch_xc_point(const XcChunkArgs& a, int count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(xc_point_kernel, dim3(a.G / 256, count), dim3(256), 0, s, a);
}

void launch_xc_reduce(const XcChunkArgs& a, int count, double* exc, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(xc_reduce_kernel, dim3(count), dim3(256), 0, s, a, exc);
}

void launch_xc_slice_sum(int n, int count, int S, const double* Vp, double* V, bool add,
                         hipStream_t s) {
  if (count == 0 || n == 0) return;
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(xc_slice_sum_kernel, dim3((unsigned)((nn + 255) / 256), count), dim3(256), 0,
                     s, n, S, Vp, V, add ? 1 : 0);
}

void launch_xc_symmetrize(int n, int count, double* V, hipStream_t s) {
  if (count == 0 || n == 0) return;
  hipLaunchKernelGGL(xc_symmetrize_kernel, dim3((n + 255) / 256, n, count), dim3(256), 0, s, n, V);
}

void launch_xc_sparse_basis(const XcSparseArgs& a, int max_nsh, hipStream_t s) {
  const int slots = a.nch * a.count;
  if (slots == 0) return;
  hipLaunchKernelGGL(xc_sparse_basis_kernel, dim3(a.G / kXcSB, max_nsh + 1, slots), dim3(kXcSB), 0, s,
                     a);
}

void launch_xc_sparse_gather(const XcSparseArgs& a, hipStream_t s) {
  const long long ww = (long long)a.W * a.W;
  const int slots = a.nch * a.count;
  if (slots == 0 || ww == 0) return;
  hipLaunchKernelGGL(xc_sparse_gather_kernel, dim3((unsigned)((ww + 255) / 256), slots), dim3(256),
                     0, s, a);
}

void launch_xc_sparse_point(const XcSparseArgs& a, hipStream_t s) {
  const int slots = a.nch * a.count;
  if (slots == 0) return;
  hipLaunchKernelGGL(xc_sparse_point_kernel, dim3(a.G / kXcSB, slots), dim3(kXcSB), 0, s, a);
}

void launch_xc_sparse_scatter(const XcSparseArgs& a, hipStream_t s) {
  const long long ww = (long long)a.W * a.W;
  const int slots = a.nch * a.count;
  if (slots == 0 || ww == 0) return;
  hipLaunchKernelGGL(xc_sparse_scatter_kernel, dim3((unsigned)((ww + 255) / 256), slots), dim3(256),
                     0, s, a);
}

void launch_xc_sparse_reduce(const XcSparseArgs& a, double* exc, hipStream_t s) {
  if (a.count == 0 || a.nch == 0) return;
  hipLaunchKernelGGL(xc_sparse_reduce_kernel, dim3(a.count), dim3(256), 0, s, a, exc);
}

void launch_xc_sparse_gpoint(const XcSparseArgs& a, double* gf, double* eg, hipStream_t s) {
  if (a.nch * a.count == 0) return;
  hipLaunchKernelGGL(xc_sparse_gpoint_kernel, dim3(a.G / kXcSB, a.nch * a.count), dim3(kXcSB), 0, s,
                     a, gf, eg);
}

void launch_xc_sparse_force(const XcSparseArgs& a, int max_nsh, const double* gf,
                            const double* Y, const int* atom_off, double* grad, hipStream_t s) {
  if (a.nch * a.count == 0 || max_nsh == 0) return;
  hipLaunchKernelGGL(xc_sparse_force_kernel, dim3(a.G / kXcSB, max_nsh, a.nch * a.count),
                     dim3(kXcSB), 0, s, a, gf, Y, atom_off, grad);
}

void launch_xc_weight_grad(const XcGridArgs& a, const double* eg, double* grad, hipStream_t s) {
  if (a.npts == 0) return;
  const size_t lds = sizeof(double) * (128 + 3) * (size_t)a.natoms;
  hipLaunchKernelGGL(xc_weight_grad_kernel, dim3((a.npts + 63) / 64), dim3(64), lds, s, a, eg,
                     grad);
}

void launch_xc_functional(int n, const double* rho, const double* sigma, double* e, double* vr,
                          double* vs, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(xc_functional_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, rho, sigma, e,
                     vr, vs);
}

}  // namespace bscf
