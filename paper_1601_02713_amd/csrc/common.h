// Shared device/host data layouts of the batched direct-SCF engine.
//
// All instances (beads, images or independent clusters) live in one set of
// flat arrays: shells, shell pairs and primitive pairs are concatenated over
// instances; n x n matrices of instance i start at moff[i] (row-major FP64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bscf {

constexpr int kLmax = 2;            // s, p, d shells
constexpr int kBoysRows = 401;      // Boys table grid T = 0, 0.1, ..., 40
constexpr double kBoysStep = 0.1;
constexpr double kBoysTmax = 40.0;  // asymptotic branch at and above
constexpr int kBoysCols = 24;       // F_0..F_22 and exp(-T_k) in column 23
constexpr int kBoysExpCol = 23;
constexpr int kWave = 64;
// XCDs of an MI355X.  The dispatcher deals the workgroups of a launch to
// them in turn by linear id, and each XCD has its own L2, so launches that
// want an instance's data to stay in one L2 place its blocks at ids
// congruent modulo kXcds.
constexpr int kXcds = 8;

// Primitive pair of a contracted shell pair (a, b) with la >= lb.
struct PrimPair {
  double p;              // alpha + beta
  double Px, Py, Pz;     // (alpha A + beta B) / p
  double PAx, PAy, PAz;  // P - A
  double C;              // sqrt(2) pi^{5/4} c_a c_b exp(-alpha beta/p |AB|^2) / p
  double oo2p;           // 1 / (2p)
  double alpha, beta;    // exponents on A and B (gradients)
  double pad;
};

struct Shell {
  double x, y, z;
  int l;
  int bf;      // first basis function, local to the instance
  int inst;
  int atom;    // global atom index
  int prim0;   // into the shell-primitive arrays
  int nprim;
};

struct ShellPair {
  int a, b;    // global shell indices, l(a) >= l(b)
  int prim0;   // first PrimPair
  int nprim;   // primitive pairs
};

// A row of the screened work list: bra shell pair `bra` against the nket ket
// pairs kets[ket0 ...] (one angular class, one primitive count, Schwarz
// prefix).  Rows of one instance and one (bra, ket) primitive-count pair are
// consecutive.
struct WorkRow {
  int bra;
  int ket0;
  int nket;
  int pad;
};

// One wavefront's work: `count` (<= 64) consecutive quartets starting at
// quartet `off` of row `row`, all of one instance and one contraction pair.
struct WorkItem {
  int row;
  int off;
  int count;
  int pad;
};

// Quartet of lane `lane` of item `it`; returns false (and a valid dummy
// quartet) for lanes beyond it.count.  `single_row` is true when the whole
// item lies in one row (uniform bra across the wavefront).
__device__ __forceinline__ bool lane_quartet(const WorkItem& it, const WorkRow* __restrict__ rows,
                                             const int* __restrict__ kets, int lane, int& bra,
                                             int& ket, bool& single_row) {
  const WorkRow r0 = rows[it.row];
  single_row = r0.nket - it.off >= it.count;
  if (lane >= it.count) {
    bra = r0.bra;
    ket = kets[r0.ket0 + it.off];
    return false;
  }
  int r = it.row, k = it.off + lane, nk = r0.nket;
  while (k >= nk) {
    k -= nk;
    ++r;
    nk = rows[r].nket;
  }
  bra = rows[r].bra;
  ket = kets[rows[r].ket0 + k];
  return true;
}

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Order-independent accumulation for the deterministic Fock build.  A value
// is held as a signed 128-bit fixed-point number with 80 fractional bits in
// two 64-bit words, p[0] = low word, p[1] = high word (two's complement).
// fx_add converts v exactly (to 2^-80) and adds it with two integer atomics,
// the carry of the low word going into the high one; integer addition is
// associative, so the total does not depend on the order of the adds, and it
// is the exact sum of the contributions.  |values| must stay below 2^47.
__device__ __forceinline__ void fx_add(unsigned long long* p, double v) {
  const double x = v * 0x1p16;
  const double h = floor(x);
  const unsigned long long lo = (unsigned long long)((x - h) * 0x1p64);
  const long long hi = (long long)h;
  const unsigned long long old = atomicAdd(p, lo);
  const long long carry = (old + lo < old) ? 1 : 0;
  if (hi + carry != 0) atomicAdd(p + 1, (unsigned long long)(hi + carry));
}

__device__ __forceinline__ double fx_value(const unsigned long long* p) {
  return (double)(long long)p[1] * 0x1p-16 + (double)p[0] * 0x1p-80;
}

}  // namespace bscf
