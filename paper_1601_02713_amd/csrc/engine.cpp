// Host side of the batched direct-SCF engine and its C ABI (include/beadscf.h).
//
// Per geometry: shell pairs and primitive pairs (device kernel), Schwarz
// bounds Q_ab = sqrt(max |(ab|ab)|) (device), screened work lists (host,
// integer work only: pairs sorted by Q per class and primitive count, each bra
// taking the surviving prefix of kets with Q_ab Q_cd >= tau, the paper's
// integral cutoff of Section 3.1), S, T, V (device) and X = S^{-1/2}.
// Per SCF iteration over all active instances: J/K by the generated class
// kernels, Fock assembly and energy, commutator error, DIIS, orthogonalised
// eigensolve and the new density, convergence flags (one device->host copy of
// per-instance flags per iteration; converged instances are masked).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <exception>
#include <fstream>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <stdexcept>
#include <string>
#include <future>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/beadscf.h"
#include "classes.h"
#include "common.h"
#include "kernels.h"
#include "grad.h"
#include "mlp.h"
#include "pimd.h"
#include "string_method.h"
#include "xc.h"

using namespace bscf;

namespace {

// quartets per lane-kernel unit: the K rows of its bra are flushed once per
// unit, so longer units amortise the flush, shorter ones spread the work
// Quartets per lane-kernel unit: 256, doubled for every doubling of the
// batch's largest basis beyond 152 functions (to 2048 at most), so that the
// unit's fixed cost, loading and flushing (n_a + n_b) rows of n elements, stays
// a like share of its integral work as n grows.
int unit_quartets(int max_n) {
  int u = 256;
  for (int n = 304; n <= max_n && u < 2048; n *= 2) u *= 2;
  return u;
}

// The HIP runtime backs a kernel's private segment with scratch reserved per
// hardware queue for full occupancy (bytes per lane x 64 lanes x 32 waves x
// 256 CUs) and keeps the reservation while the process lives; several
// contexts in one process reach several queues.  Lane kernels that spill more
// than this many bytes per lane are never launched (their class runs
// cooperatively), which bounds every queue's reservation to about 2 GiB of
// the 288 GB; below it the autotuner times both forms and keeps the faster.
constexpr int kMaxLaneScratch = 4096;

// The bound a context applies: kMaxLaneScratch, or less when the environment
// variable BSCF_LANE_SCRATCH_MAX asks for less (tests use it to route classes
// whose lane kernels spill less than kMaxLaneScratch to the cooperative form).
int lane_scratch_bound() {
  const char* v = getenv("BSCF_LANE_SCRATCH_MAX");
  if (!v || !*v) return kMaxLaneScratch;
  return std::max(0, std::min(kMaxLaneScratch, atoi(v)));
}

// Incremental Fock builds: a full build at the first SCF iteration and every
// kFullEvery iterations, which bounds the accumulated effect of the skipped
// quartets.  Their sum (each below the cutoff, over millions of quartets in
// a large instance) also puts a floor under the commutator error, near 1e-8
// for 608 functions: once an instance within kStallNear times comm_tol has
// not brought its error below kStallRatio of its value two iterations back
// (at least two iterations after a full build), the rest of the SCF call
// builds in full.
constexpr int kFullEvery = 12;
constexpr double kStallNear = 100.0;
constexpr double kStallRatio = 0.8;

// SP2 purification: at most kSp2MaxSteps projection steps per density; a
// replica's projector counts as converged once the idempotency error
// Tr X - Tr X^2 = sum_k l_k (1 - l_k) is below kSp2Tol and Tr X is N/2 within
// kSp2TraceTol (two more steps then square the residual occupation error
// away).  A call launches the step count the last call needed plus
// kSp2Margin before it looks at the result; steps past a replica's need are
// copies.
constexpr int kSp2MaxSteps = 100;
constexpr double kSp2Tol = 1e-11;
constexpr double kSp2TraceTol = 1e-6;
constexpr int kSp2Margin = 4;

thread_local std::string g_err;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw Error(BSCF_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)
#define BLASCHK(x)                                                                        \
  do {                                                                                    \
    rocblas_status s_ = (x);                                                              \
    if (s_ != rocblas_status_success)                                                     \
      throw Error(BSCF_E_DEVICE, std::string(#x) + ": rocblas status " + std::to_string(s_)); \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void resize(size_t m) {
    if (m <= n && p) return;
    release();
    if (m == 0) m = 1;
    if (hipMalloc(&p, m * sizeof(T)) != hipSuccess) {
      p = nullptr;
      throw Error(BSCF_E_NOMEM, "hipMalloc of " + std::to_string(m * sizeof(T)) + " bytes failed");
    }
    n = m;
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    resize(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// Pinned host memory (hipHostMalloc) for the small device-to-host reads the
// SCF loop waits on.
template <typename T>
struct PinBuf {
  T* p = nullptr;
  size_t n = 0;
  PinBuf() = default;
  PinBuf(const PinBuf&) = delete;
  PinBuf& operator=(const PinBuf&) = delete;
  ~PinBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  void resize(size_t m) {
    if (m <= n && p) return;
    release();
    if (m == 0) m = 1;
    if (hipHostMalloc((void**)&p, m * sizeof(T), hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      throw Error(BSCF_E_NOMEM, "hipHostMalloc of " + std::to_string(m * sizeof(T)) + " bytes failed");
    }
    n = m;
  }
};

// ------------------------------------------------------------ mini JSON
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const std::string& k) const {
    for (auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* s;
  void ws() { while (*s && isspace((unsigned char)*s)) ++s; }
  [[noreturn]] void fail(const char* m) { throw Error(BSCF_E_INVALID, std::string("basis JSON: ") + m); }
  JVal parse() {
    ws();
    JVal v;
    if (*s == '{') {
      v.kind = JVal::OBJ;
      ++s;
      ws();
      if (*s == '}') { ++s; return v; }
      for (;;) {
        ws();
        if (*s != '"') fail("expected key");
        std::string k = str();
        ws();
        if (*s != ':') fail("expected ':'");
        ++s;
        v.obj.emplace_back(k, parse());
        ws();
        if (*s == ',') { ++s; continue; }
        if (*s == '}') { ++s; return v; }
        fail("expected ',' or '}'");
      }
    } else if (*s == '[') {
      v.kind = JVal::ARR;
      ++s;
      ws();
      if (*s == ']') { ++s; return v; }
      for (;;) {
        v.arr.push_back(parse());
        ws();
        if (*s == ',') { ++s; continue; }
        if (*s == ']') { ++s; return v; }
        fail("expected ',' or ']'");
      }
    } else if (*s == '"') {
      v.kind = JVal::STR;
      v.str = str();
    } else if (!strncmp(s, "true", 4)) {
      v.kind = JVal::BOOL; v.num = 1; s += 4;
    } else if (!strncmp(s, "false", 5)) {
      v.kind = JVal::BOOL; s += 5;
    } else if (!strncmp(s, "null", 4)) {
      s += 4;
    } else {
      char* end;
      v.num = strtod(s, &end);
      if (end == s) fail("bad value");
      v.kind = JVal::NUM;
      s = end;
    }
    return v;
  }
  std::string str() {
    std::string out;
    ++s;
    while (*s && *s != '"') {
      if (*s == '\\' && s[1]) { out.push_back(s[1]); s += 2; continue; }
      out.push_back(*s++);
    }
    if (*s != '"') fail("unterminated string");
    ++s;
    return out;
  }
};

struct BasisShell {
  int l;
  std::vector<double> exps, coefs;  // coefs: d_k * radial norm * contraction rescale
};

// radial primitive normalisation (2a/pi)^{3/4} (4a)^{l/2}, the x^l component
// carrying the double factorial separately; the contraction is rescaled so that
// <phi|phi> = 1 with <g_i|g_j> = (pi/(ai+aj))^{3/2} (2l-1)!!/(2(ai+aj))^l.
BasisShell normalise_shell(int l, const std::vector<double>& e, const std::vector<double>& d) {
  BasisShell s;
  s.l = l;
  s.exps = e;
  const double pi = M_PI;
  std::vector<double> c(e.size());
  for (size_t k = 0; k < e.size(); ++k)
    c[k] = d[k] * std::pow(2.0 * e[k] / pi, 0.75) * std::pow(4.0 * e[k], 0.5 * l);
  double dfac = 1.0;
  for (int k = 2 * l - 1; k > 1; k -= 2) dfac *= k;
  double ss = 0.0;
  for (size_t i = 0; i < e.size(); ++i)
    for (size_t j = 0; j < e.size(); ++j) {
      const double p = e[i] + e[j];
      ss += c[i] * c[j] * std::pow(pi / p, 1.5) * dfac / std::pow(2.0 * p, l);
    }
  // the component norm 1/sqrt((2l-1)!!) of x^l makes the self-overlap ss/dfac
  const double r = 1.0 / std::sqrt(ss / dfac);
  for (auto& x : c) x *= r;
  s.coefs = c;
  return s;
}

struct Group {
  int first, count, n;
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct bscf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  static constexpr int kAux = 4;   // streams for concurrent class kernels
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
  // profiling: event pairs recorded around launches and read back only when
  // the statistics are requested, so the timed work is not synchronised
  struct ProfRec {
    hipEvent_t e0, e1;
    int q, kind;   // class index; kind: 0 Fock class kernel, 1 gradient class kernel, 2 whole
                   // build, 3 exchange-correlation step q (XcStep)
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_free;
  // Kernel variant per class: 0 = one quartet per lane, 1 = one quartet per
  // wavefront (cooperative); [precision mode][class] for the Fock build and
  // [class] for the gradient.  Chosen by timing both on the current work
  // lists (autotune) unless BSCF_VARIANT=lane|coop forces one.
  int fock_variant[2][kNumQuartetClasses] = {};
  int grad_variant[kNumQuartetClasses] = {};
  bool fock_tuned[2] = {false, false};
  bool grad_tuned = false;
  // fock_variant[precision][class]: 0 lane (MIXED: the mixed form), 1 cooperative,
  // 2 (MIXED only) the FP64 lane form; tune_ms holds their times
  float tune_ms[2][kNumQuartetClasses][3] = {};
  // threads per lane-kernel unit, [precision mode][class][variant] (see tune_ms)
  int unit_threads[2][kNumQuartetClasses][3] = {};
  float tune_grad_ms[kNumQuartetClasses][2] = {};
  int grad_unit_threads[kNumQuartetClasses] = {};   // threads per lane gradient unit
  float tune_grad1e_ms[kNumPairClasses] = {};   // one-electron gradient kernels alone
  // per-lane private (scratch) bytes of every class kernel: [class][fp64, mixed, grad].
  // The runtime reserves (and keeps) scratch per hardware queue for full
  // occupancy, so every kernel that uses scratch (class kernels, one-electron
  // and Schwarz kernels) runs on the context's own stream; only scratch-free
  // class kernels overlap on the auxiliary streams.
  int private_bytes[kNumQuartetClasses][3] = {};
  int lane_scratch_max = lane_scratch_bound();   // lane kernels above it never run
  int coop_bytes[kNumQuartetClasses][2] = {};   // cooperative fock, gradient
  double t_fock_gpu_ms = 0, t_work_ms = 0;
  // exchange-correlation builds: kernel time per step (HIP events, with
  // profiling), launches, builds, grid points evaluated and GEMM FLOPs
  double xc_ms[7] = {}, xc_points = 0, xc_gemm_flops = 0;
  // algorithmic bytes of the basis and point steps: per point 8 m + 32 and
  // 16 m + 32 with m the functions the point takes (n dense, a chunk's ns sparse)
  double xc_basis_bytes = 0, xc_point_bytes = 0;
  long long xc_launches[7] = {}, xc_builds = 0;
  double t_work_host_ms = 0;   // host part of the work lists, wherever it ran
  bool items_all = false;      // build every class's cooperative items (see build_work_host)
  double t_work_phase_ms[3] = {0, 0, 0};   // its ket lists, parts, merges
  rocblas_handle blas = nullptr;

  std::map<int, std::vector<BasisShell>> basis;

  // instances
  int ninst = 0;
  std::vector<int> natoms, atom_off, Zs, charge, nbf, nocc, nshell, shell_off;
  std::vector<long long> moff;
  long long mtot = 0;
  int max_n = 0, max_atoms = 0, total_atoms = 0;
  std::vector<Group> groups;
  // shells, pairs (topology fixed per batch composition)
  std::vector<Shell> shells;
  std::vector<double> sh_exp, sh_coef;
  std::vector<ShellPair> pairs;
  std::vector<int> pair_class;     // 0..5
  std::vector<int> prim_owner;
  int nprim_pairs = 0;
  std::vector<std::vector<int>> pairs_by_class;  // global pair ids per pair class
  std::vector<double> xyz;
  std::vector<int> atom_bf0, atom_nbf;   // per global atom: first basis function, count
  bool have_geom = false, have_scf = false;
  std::vector<double> Q;           // per pair
  double work_tau = -1.0, work_split = -1.0;   // parameters of the lists on the device
  // host lists made by build_work_host (possibly on a worker thread started by
  // bscf_set_geometries) and not yet uploaded: their parameters, ket-order
  // primitive map and positions
  double host_tau = -1.0, host_split = -1.0;
  std::future<void> work_job;
  std::vector<int2> h_kpos;
  std::vector<int> h_kmap;
  double split_tol = 1e-4;   // FP32 split of MIXED builds (from the last SCF options)
  // work lists per quartet class
  struct ClassWork {
    // 64-quartet items over rows grouped by primitive counts (cooperative
    // kernels, gradient) and per-bra units over rows grouped by bra (lane
    // Fock kernels)
    std::vector<WorkItem> items;
    std::vector<WorkRow> rows;
    DevBuf<WorkItem> d_items;
    DevBuf<WorkRow> d_rows;
    int max_prims = 1;   // largest primitive count of the class's bra pairs (sizes unit LDS)
    // per-bra units over every screened quartet; each row's pad is its FP64
    // prefix, the kets with Q_ab Q_cd at or above the FP32 split of MIXED mode
    struct UnitList {
      std::vector<WorkItem> units;
      std::vector<WorkRow> rows;
      DevBuf<WorkItem> d_units;
      DevBuf<WorkRow> d_rows;
      DevBuf<int> d_keep;   // kets per row that an incremental build keeps
    } ul;
    double nquart32 = 0;                 // quartets below the FP32 split
    std::vector<double> inst_quart32;    // per instance
    double done_quart32 = 0;
    bool lds_ok = true;   // the lane kernel's LDS rows fit one workgroup
    double nquart = 0, nprimq = 0;
    std::vector<double> inst_quart, inst_primq;  // per instance
    // evaluated so far (active instances only) and measured kernel time
    double done_quart = 0, done_primq = 0, kernel_ms = 0, grad_ms = 0;
    double grad_quart = 0, grad_primq = 0;   // evaluated by the gradient (device counts)
    bool has_work = false;       // any screened quartet in the batch
    bool items_skipped = false;  // the cooperative items were not built (see build_work_host)
    // Schwarz-screened quartets (at the build's cutoff) of the instances each
    // build covered, whether a full or an incremental build evaluated them
    double screened_quart = 0;
    long launches = 0, grad_launches = 0;
  };
  ClassWork work[kNumQuartetClasses];
  std::vector<int> kets;
  DevBuf<int> d_kets;
  // ket-list-position buffers: P gathered per ket pair and ket-side J
  DevBuf<double> d_Pk, d_Jk;
  // deterministic builds: J, K and Jk in fixed point (two words per element),
  // allocated on first use; det is the setting of bscf_set_deterministic,
  // det_now that of the build in progress
  DevBuf<unsigned long long> Jfx, Kfx, Jkfx;
  bool det = false, det_now = false;
  // ket primitive pairs copied into ket-list order: within a block of
  // positions sharing a primitive count, primitive j of every position is
  // adjacent to that of the next position (coalesced lane loads)
  DevBuf<PrimPair> d_kprims;
  DevBuf<int> d_kmap;          // source primitive pair of each kprims record
  DevBuf<int2> d_kpos;         // per position: first record, stride
  int max_prims = 1;
  int max_prims_pc[kNumPairClasses] = {};   // the same per pair class
  int max_ncd = 0;
  size_t max_lds_bytes = 65536;

  // device data
  DevBuf<Shell> d_shells;
  DevBuf<double> d_sh_exp, d_sh_coef;
  DevBuf<ShellPair> d_pairs;
  DevBuf<int> d_prim_owner;
  DevBuf<PrimPair> d_prims;
  DevBuf<double> d_Q;
  std::vector<DevBuf<int>> d_pair_ids;   // per pair class
  DevBuf<double> d_boys64;
  DevBuf<float> d_boys32;
  DevBuf<int> d_nocc, d_nbf, d_natoms, d_atom_off, d_active, d_all_active, d_conv_iter, d_status;
  DevBuf<int> d_shell_off, d_nshell;     // per instance
  DevBuf<long long> d_pm_off;            // per instance: offset of its shell-block max |P|
  DevBuf<double> d_pmax;                 // [sum nsh^2] largest |P| per shell block
  DevBuf<double> d_dpm;                  // the same of the density change (incremental builds)
  int max_nshell = 0;
  DevBuf<long long> d_moff;
  DevBuf<double> d_xyz, d_Zd, d_Enuc, d_E, d_Eprev, d_emax, d_grad;
  DevBuf<double> d_grad_tune;   // [3 total_atoms]: the gradient kernels' timing pass writes here
  DevBuf<int> d_task_a, d_task_b;  // 1e tasks: pair shells
  std::vector<double> pair_rcut;    // per pair of c->pairs: distance beyond which it is negligible
  std::vector<int> task_first, task_count;  // per pair class ranges into task arrays
  // matrices
  DevBuf<double> S, T, V, H, X, F, J, K, P, Pnew, W, tmp1, tmp2, err, Fbar, C, Cacc, eig, eigE;
  // orbitals of the SCF before the last (extrapolated guess), its work buffers,
  // and per instance the number of SCFs whose orbitals are stored (0, 1, 2)
  DevBuf<double> Cprev, Cext, Mpol;
  DevBuf<int> d_cfirst, d_c2ok;
  std::vector<int> h_ccount;
  DevBuf<double> d_gstat;   // [class][2] gradient work of one forces call
  DevBuf<double> Pprev, dP, d_dpmax;   // incremental builds: last build's P, its change, max |dP|
  // work kept by incremental builds, [quartets, primitive quartets, FP32
  // quartets][class][instance], accumulated on the device until read
  DevBuf<double> d_kept;
  long long inc_builds = 0;
  DevBuf<double> Fhist, Ehist, diisB, diisC;
  DevBuf<int> diis_count, diis_head, d_info;
  // SP2 purification: per-step (Tr X, Tr X^2) of every instance, Gershgorin
  // bounds, the first converged step of every instance (two alternating
  // arrays of ninst), and the orbital-commit mask.  sp2_pred[0] is the step
  // count the last core guess needed; sp2_pred[1 + it] that of SCF iteration
  // it (the need falls over an SCF run, and runs of one batch repeat the
  // pattern); iterations past the table use its last entry
  static constexpr int kSp2PredIters = 64;
  DevBuf<double> d_sp2, d_sp2b;
  DevBuf<int> d_sp2c, d_omask;
  int sp2_pred[1 + kSp2PredIters] = {};
  long long sp2_calls = 0, sp2_steps = 0, sp2_needed = 0, sp2_fallbacks = 0;
  // what the SCF loop reads once per iteration: [ninst] active flags, then
  // [ninst] SP2 first converged steps; packed on the device, then one copy
  DevBuf<int> d_pin;
  PinBuf<int> h_pin;
  PinBuf<double> h_emax;   // the commutator errors of the last iteration
  DevBuf<double> d_wmin;    // smallest overlap eigenvalue per instance
  PinBuf<double> h_wmin;
  // captured density halves of an SCF iteration, by (SP2 steps, e_tol,
  // comm_tol, DIIS size); they hold device addresses of this context's
  // buffers, so every change of the batch drops them
  std::map<std::tuple<int, double, double, int>, hipGraphExec_t> graphs;
  long long graph_launches = 0, graph_captures = 0;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
    drop_fock_graphs();
  }
  // J and K accumulation of Fock builds captured as graphs (bscf_scf_opts
  // graph 2), per (precision, masked, incremental, deterministic, tau); they
  // hold the addresses and launch shapes of the work lists and the tuned
  // kernels, so every change of those drops them
  std::map<std::tuple<int, int, int, int, double>, hipGraphExec_t> fock_graphs;
  int graph_fock = 0;
  long long fock_graph_launches = 0, fock_graph_captures = 0, graph_memset_nodes = 0;
  void drop_fock_graphs() {
    for (auto& g : fock_graphs) (void)hipGraphExecDestroy(g.second);
    fock_graphs.clear();
  }
  bool have_C = false;
  std::vector<int> h_active;   // host copy of the active flags
  bool profiling = false;

  // stats
  double t_fock_ms = 0, t_scf_ms = 0, t_grad_ms = 0, t_setup_ms = 0;
  int fock_builds = 0, scf_iters = 0;
  std::vector<int> last_iters;

  mlp::Guess guess;

  // ring-polymer integrator over the batch's instances (its beads); state on
  // the device between steps
  struct Pimd {
    bool on = false;
    int P = 0, N = 0;
    bscf_pimd_opts o{};
    uint64_t step = 0;
    bool synced = false;       // the context's geometry is the integrator's positions
    bool have_force = false;   // d_grad holds the gradient at the current positions
    DevBuf<double> x, p, C, w, c1, c2, mass, sig, F;
  } md;

  // B3LYP exchange-correlation: xc the setting of bscf_set_xc, xc_now that of
  // the build in progress, scf_xc that of the last SCF (its forces add the XC term)
  int xc = 0, xc_now = 0;
  bool scf_xc = false;
  struct Xcs {
    bool tables = false;
    bool grid_ok = false;               // the grid of the current geometry is on the device
    std::vector<long long> pt_off;      // per instance: first grid point
    std::vector<int> npts_i;            // per instance: grid points
    long long npts = 0;
    DevBuf<double> rad_r, rad_w, ang_u, ang_w, pts;
    DevBuf<long long> d_pt_off;
    DevBuf<int> d_npts, d_sh_off, d_nsh;
    DevBuf<double> B, Z, part;          // chunk buffers [count][n][G], partial sums
    DevBuf<double> Vp;                  // [count][S][n][n] slice products
    DevBuf<double*> gp;                 // slice GEMM operands: A, B, C pointer arrays
    std::vector<double*> hgp;
    // sparse form, per group (xc.h): chunks of kXcSparseShells radial shells
    // of one atom and the basis shells each takes
    struct Chunk {
      int p0, gcnt, sh0, nsh, f0, ns, sec;
    };
    // chunks of similar size share a launch, padded to W functions
    struct Bucket {
      int c0, nch, W, max_nsh;   // chunks [c0, c0 + nch) of the group's sorted list
    };
    struct GroupChunks {
      bool sparse = false;
      std::vector<Chunk> chunks;   // largest first
      std::vector<Bucket> buckets;
      int meta0 = 0;               // first chunk's entry in d_meta
    };
    std::vector<GroupChunks> gch;
    std::vector<double> h_rad_r;        // [2][kXcRad] radial points (H, others)
    DevBuf<int> d_shl, d_scbf, d_fmap;  // the chunks' shell lists, compact offsets, function maps
    DevBuf<int> d_meta;                 // [chunk][kXcMeta] of every group's sorted chunks
    DevBuf<int> d_sec_ang;              // [kXcSectors][kXcSectorAng] angular nodes per sector
    std::vector<double> h_ang_u;        // [kXcAng][3] directions (host copy)
    DevBuf<double> Ps, Vs;
    DevBuf<double> V, exc;              // V_xc [mtot], E_xc [ninst]
    // gradient (xc.h): Y = D Ps per slot, the point factors, e per grid point
    DevBuf<double> Yg, gf, eg;
    DevBuf<double> isep;                // per instance [natoms][natoms] 1/|R_A - R_B|
    std::vector<long long> isep_off;
  } xcs;

  // string of images over the batch's instances; positions on the device
  struct Str {
    bool on = false;
    int n = 0, N = 0;
    bscf_string_opts o{};
    bool synced = false;   // the context's geometry is the images' positions
    long long iters = 0;
    DevBuf<double> x, xt, F, arc;
  } str;

  BatchInfo batch(bool masked) const {
    BatchInfo b;
    b.ninst = ninst;
    b.nbf = d_nbf.p;
    b.moff = d_moff.p;
    b.active = masked ? d_active.p : nullptr;
    return b;
  }
};

namespace {

template <typename F>
bscf_status guard(F&& f) {
  try {
    f();
    g_err.clear();
    return BSCF_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_err = e.what();
    return BSCF_E_DEVICE;
  }
}

void need(bool c, int code, const std::string& m) {
  if (!c) throw Error(code, m);
}

// pair class index of (la, lb), la >= lb: ss, ps, pp, ds, dp, dd
int pclass(int la, int lb) { return la * (la + 1) / 2 + lb; }

void sync(bscf_ctx* c) { HIPCHK(hipStreamSynchronize(c->stream)); }

// ---- dense helpers over groups of equal-n consecutive instances
void gemm(bscf_ctx* c, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
          double alpha, const double* A, const double* B, double beta, double* Cm) {
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int mm = m < 0 ? g.n : m, nn = n < 0 ? g.n : n, kk = k < 0 ? g.n : k;
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, ta, tb, mm, nn, kk, &alpha, A + o, g.n, st,
                                          B + o, g.n, st, &beta, Cm + o, g.n, st, g.count));
  }
}

// symmetric eigendecomposition in place: A <- eigenvectors (columns), w <- values
void syevd(bscf_ctx* c, double* A, double* w) {
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    // eigenvalues of instance i stored at w + moff[i] (row 0 of its block)
    BLASCHK(rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper,
                                             g.n, A + o, g.n, st, w + o, st, c->eigE.p + o, st,
                                             c->d_info.p + g.first, g.count));
  }
}

__global__ void scale_cols_kernel(BatchInfo b, const double* U, const double* w, double* out,
                                  double power) {
  const int inst = blockIdx.y;
  const int n = b.nbf[inst];
  const long long o = b.moff[inst], nn = (long long)n * n;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    const long long col = k / n;  // column-major: element k = (row k%n, col k/n)
    out[o + k] = U[o + k] * pow(w[o + col], power);
  }
}

__global__ void min_eig_kernel(BatchInfo b, const double* w, double* out) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= b.ninst) return;
  out[inst] = w[b.moff[inst]];
}

// X = S^{-1/2} (Loewdin) for every instance
void build_orthogonaliser(bscf_ctx* c) {
  const long long mt = c->mtot;
  HIPCHK(hipMemcpyAsync(c->eig.p, c->S.p, mt * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  syevd(c, c->eig.p, c->tmp2.p);
  // smallest eigenvalue check (gathered on the device, one read)
  BatchInfo b = c->batch(false);
  hipLaunchKernelGGL(min_eig_kernel, dim3((c->ninst + 63) / 64), dim3(64), 0, c->stream, b,
                     c->tmp2.p, c->d_wmin.p);
  HIPCHK(hipMemcpyAsync(c->h_wmin.p, c->d_wmin.p, c->ninst * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  sync(c);
  for (int i = 0; i < c->ninst; ++i)
    need(c->h_wmin.p[i] > 1e-7, BSCF_E_UNSUPPORTED,
         "overlap matrix of instance " + std::to_string(i) + " is near-singular (min eigenvalue " +
             std::to_string(c->h_wmin.p[i]) + ")");
  const long long nn = (long long)c->max_n * c->max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(scale_cols_kernel, dim3(gx, c->ninst), dim3(256), 0, c->stream, b, c->eig.p,
                     c->tmp2.p, c->tmp1.p, -0.5);
  // X = (U w^{-1/2}) U^T
  gemm(c, rocblas_operation_none, rocblas_operation_transpose, -1, -1, -1, 1.0, c->tmp1.p,
       c->eig.p, 0.0, c->X.p);
}

// orthonormal-basis Fock matrix F' = X Fb X into eig
void ortho_fock(bscf_ctx* c, const double* Fb) {
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->X.p, Fb, 0.0,
       c->tmp1.p);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->tmp1.p, c->X.p, 0.0,
       c->eig.p);
}

// orbitals of Fb: eig <- eigenvectors of F' = X Fb X, C = X C'
void orbitals_from_fock(bscf_ctx* c, const double* Fb) {
  ortho_fock(c, Fb);
  syevd(c, c->eig.p, c->tmp2.p);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->X.p, c->eig.p, 0.0,
       c->C.p);
}

// P = 2 C_occ C_occ^T from the orbitals in C
void density_from_orbitals(bscf_ctx* c, double* Pout) {
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int no = c->nocc[g.first];
    const double two = 2.0, zero = 0.0;
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                          rocblas_operation_transpose, g.n, g.n, no, &two,
                                          c->C.p + o, g.n, st, c->C.p + o, g.n, st, &zero,
                                          Pout + o, g.n, st, g.count));
  }
}

// SP2 on F' (in eig) for the instances of the device mask of b.  X_k
// alternates between tmp1 and tmp2, each step one fused product-and-update
// launch that also decides, per instance, when the projection is finished
// (launch_sp2_step); the first converged step of instance i after k steps is
// at d_sp2c[(k & 1) * ninst + i].
void sp2_start(bscf_ctx* c, const BatchInfo& b) {
  launch_sp2_bounds(b, c->max_n, c->eig.p, c->d_sp2b.p, c->stream);
  launch_sp2_init(b, c->max_n, c->eig.p, c->d_sp2b.p, c->tmp1.p, c->d_sp2.p, c->d_sp2c.p,
                  c->stream);
}

// steps k0 .. k1 - 1
void sp2_steps(bscf_ctx* c, const BatchInfo& b, int k0, int k1) {
  const long long row = 2LL * c->ninst * sp2_tiles(c->max_n);   // statistics of one step
  double* buf[2] = {c->tmp1.p, c->tmp2.p};
  for (int k = k0; k < k1; ++k)
    launch_sp2_step(b, c->max_n, c->d_nocc.p, buf[k & 1], buf[(k + 1) & 1], c->d_sp2.p + k * row,
                    c->d_sp2.p + (k + 1) * row, k, kSp2Tol, kSp2TraceTol,
                    c->d_sp2c.p + (k & 1) * c->ninst, c->d_sp2c.p + ((k + 1) & 1) * c->ninst,
                    c->stream);
}

// P = 2 X X_k X into Pout
void sp2_project(bscf_ctx* c, int k, double* Pout) {
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->X.p,
       (k & 1) ? c->tmp2.p : c->tmp1.p, 0.0, c->eig.p);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 2.0, c->eig.p, c->X.p, 0.0,
       Pout);
}

// Step predictor index: the core guess, or SCF iteration it.
int sp2_slot(int it) { return it < 0 ? 0 : 1 + std::min(it, bscf_ctx::kSp2PredIters - 1); }

// Steps to launch ahead for predictor slot which: its last need (or, where
// that has no record yet, that of an earlier slot) plus a margin.
int sp2_target(bscf_ctx* c, int which) {
  int pred = 0;
  for (int w = which; w >= 0 && pred == 0; --w) pred = c->sp2_pred[w];
  if (pred == 0) pred = 48;
  return std::min(pred + kSp2Margin, kSp2MaxSteps);
}

// Launch a whole SP2 density of k steps without waiting, then the projector
// into Pout.
void sp2_launch(bscf_ctx* c, const BatchInfo& b, int k, double* Pout) {
  sp2_start(c, b);
  sp2_steps(c, b, 0, k);
  sp2_project(c, k, Pout);
}

// Queue the read of the first converged steps after k steps into h_pin[ninst..].
void sp2_read(bscf_ctx* c, int k) {
  HIPCHK(hipMemcpyAsync(c->h_pin.p + c->ninst, c->d_sp2c.p + (k & 1) * c->ninst,
                        c->ninst * sizeof(int), hipMemcpyDeviceToHost, c->stream));
}

// After sp2_read(c, k) and a synchronisation: true when every instance of
// act finished within k steps (then sp2_pred[which] becomes the largest need).
bool sp2_finished(bscf_ctx* c, const std::vector<int>& act, int k, int which) {
  const int* first = c->h_pin.p + c->ninst;
  int need = 0;
  for (int i = 0; i < c->ninst; ++i) {
    if (!act[i]) continue;
    if (first[i] < 0 || first[i] + 2 > k) return false;
    need = std::max(need, first[i] + 2);
  }
  if (need > 0) {
    c->sp2_pred[which] = need;
    c->sp2_needed += need;
  }
  return true;
}

// Continue a projection that has not finished after k steps, in batches of a
// quarter of the steps so far (at least 4) with a check after each; on
// success the projector goes to Pout.  False when some instance of act has
// not converged after kSp2MaxSteps (no gap).  k is updated to the steps
// launched.
bool sp2_extend(bscf_ctx* c, const BatchInfo& b, const std::vector<int>& act, int which, int& k,
                double* Pout) {
  while (k < kSp2MaxSteps) {
    const int k1 = std::min(k + std::max(4, k / 4), kSp2MaxSteps);
    sp2_steps(c, b, k, k1);
    k = k1;
    sp2_read(c, k);
    sync(c);
    if (sp2_finished(c, act, k, which)) {
      sp2_project(c, k, Pout);
      return true;
    }
  }
  return false;
}

// SP2 density of the instances with act[i] set (the device mask of b
// matches), waiting for the result; which selects the step predictor.  False
// when some has not converged after kSp2MaxSteps steps.
bool density_sp2(bscf_ctx* c, const BatchInfo& b, const std::vector<int>& act, int which,
                 double* Pout) {
  int k = sp2_target(c, which);
  sp2_launch(c, b, k, Pout);
  sp2_read(c, k);
  sync(c);
  const bool ok = sp2_finished(c, act, k, which) || sp2_extend(c, b, act, which, k, Pout);
  c->sp2_calls++;
  c->sp2_steps += k;
  return ok;
}

// density of the Fock matrix Fb (the core Hamiltonian of a guess) for the
// replicas with act[i] (device mask of b): SP2 by default, the eigenvector
// route on request or when SP2 finds no gap
void density_from_fock(bscf_ctx* c, const double* Fb, const BatchInfo& b,
                       const std::vector<int>& act, int method, double* Pout) {
  if (method == BSCF_DENSITY_SP2) {
    ortho_fock(c, Fb);
    if (density_sp2(c, b, act, sp2_slot(-1), Pout)) return;
    c->sp2_fallbacks++;
  }
  orbitals_from_fock(c, Fb);
  density_from_orbitals(c, Pout);
}

// The steps of one SCF iteration after its Fock build: the commutator error
// e = X (FPS - SPF) X, the convergence test, DIIS, the density of the
// extrapolated F (SP2 with k steps, or the eigenvector route when k < 0) and
// its commit, and the packing of what the host reads afterwards.  DIIS, the
// density and the commit follow the device's active flags, so this runs
// before the host knows which replicas the test has just finished.  Every
// launch argument is a buffer of the context or a value fixed for the SCF
// call, so with SP2 the sequence is the same for every iteration of k steps.
void density_half(bscf_ctx* c, const bscf_scf_opts& o, const DiisArgs& d, const BatchInfo& bm,
                  int k) {
  const hipStream_t st = c->stream;
  const int ni = c->ninst;
  // M = F P S, e = X (M - M^T) X
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->F.p, c->P.p, 0.0,
       c->tmp1.p);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->tmp1.p, c->S.p, 0.0,
       c->tmp2.p);
  launch_antisym(c->batch(false), c->max_n, c->tmp2.p, c->tmp1.p, c->d_emax.p, st);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->X.p, c->tmp1.p, 0.0,
       c->tmp2.p);
  gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->tmp2.p, c->X.p, 0.0,
       c->err.p);
  launch_convergence(ni, c->max_n, c->d_nbf.p, c->d_E.p, c->d_Eprev.p, c->d_emax.p, o.e_tol,
                     o.comm_tol, c->d_active.p, c->d_conv_iter.p, c->d_status.p, st);
  launch_diis_store(d, c->max_n, c->F.p, c->err.p, st);
  launch_diis_extrapolate(d, c->max_n, c->Fbar.p, st);
  if (k >= 0) {
    ortho_fock(c, c->Fbar.p);
    sp2_launch(c, bm, k, c->Pnew.p);
  } else {
    orbitals_from_fock(c, c->Fbar.p);
    density_from_orbitals(c, c->Pnew.p);
  }
  launch_commit(bm, c->max_n, c->Pnew.p, c->P.p, st);
  launch_concat_ints(c->d_active.p, ni, k >= 0 ? c->d_sp2c.p + (k & 1) * ni : nullptr,
                     k >= 0 ? ni : 0, c->d_pin.p, st);
}

// memset nodes of a captured graph (library calls can record them; the
// statistics report them so that tests can insist on none)
int memset_nodes(hipGraph_t g) {
  size_t n = 0;
  HIPCHK(hipGraphGetNodes(g, nullptr, &n));
  std::vector<hipGraphNode_t> nodes(n);
  if (n) HIPCHK(hipGraphGetNodes(g, nodes.data(), &n));
  int k = 0;
  for (hipGraphNode_t v : nodes) {
    hipGraphNodeType t;
    HIPCHK(hipGraphNodeGetType(v, &t));
    if (t == hipGraphNodeTypeMemset) ++k;
  }
  return k;
}

// density_half with SP2 of k steps as one launch of a HIP graph, captured
// from the same calls the first time this (k, tolerances, DIIS size) occurs.
void density_half_graph(bscf_ctx* c, const bscf_scf_opts& o, const DiisArgs& d,
                        const BatchInfo& bm, int k) {
  const auto key = std::make_tuple(k, o.e_tol, o.comm_tol, o.diis_size);
  auto g = c->graphs.find(key);
  if (g == c->graphs.end()) {
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t graph = nullptr;
    try {
      density_half(c, o, d, bm, k);
    } catch (...) {
      (void)hipStreamEndCapture(c->stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    HIPCHK(hipStreamEndCapture(c->stream, &graph));
    c->graph_memset_nodes += memset_nodes(graph);
    hipGraphExec_t exec = nullptr;
    const hipError_t r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(r);
    g = c->graphs.emplace(key, exec).first;
    c->graph_captures++;
  }
  HIPCHK(hipGraphLaunch(g->second, c->stream));
  c->graph_launches++;
}

void build_shell_topology(bscf_ctx* c) {
  c->shells.clear();
  c->sh_exp.clear();
  c->sh_coef.clear();
  c->pairs.clear();
  c->pair_class.clear();
  c->prim_owner.clear();
  c->nshell.assign(c->ninst, 0);
  c->shell_off.assign(c->ninst, 0);
  c->pairs_by_class.assign(kNumPairClasses, {});
  c->atom_bf0.assign(c->total_atoms, 0);
  c->atom_nbf.assign(c->total_atoms, 0);
  for (int i = 0; i < c->ninst; ++i) {
    c->shell_off[i] = (int)c->shells.size();
    int bf = 0;
    for (int a = 0; a < c->natoms[i]; ++a) {
      const int z = c->Zs[c->atom_off[i] + a];
      for (const BasisShell& bs : c->basis[z]) {
        Shell s{};
        s.l = bs.l;
        s.bf = bf;
        s.inst = i;
        s.atom = c->atom_off[i] + a;
        s.prim0 = (int)c->sh_exp.size();
        s.nprim = (int)bs.exps.size();
        for (size_t k = 0; k < bs.exps.size(); ++k) {
          c->sh_exp.push_back(bs.exps[k]);
          c->sh_coef.push_back(bs.coefs[k]);
        }
        if (c->atom_nbf[s.atom] == 0) c->atom_bf0[s.atom] = bf;
        c->atom_nbf[s.atom] += ncart(bs.l);
        bf += ncart(bs.l);
        c->shells.push_back(s);
      }
    }
    c->nshell[i] = (int)c->shells.size() - c->shell_off[i];
    // pairs a >= b (index), stored with the higher l first
    const int s0 = c->shell_off[i], ns = c->nshell[i];
    for (int a = 0; a < ns; ++a)
      for (int b = 0; b <= a; ++b) {
        int sa = s0 + a, sb = s0 + b;
        if (c->shells[sa].l < c->shells[sb].l) std::swap(sa, sb);
        ShellPair p;
        p.a = sa;
        p.b = sb;
        p.prim0 = c->nprim_pairs;
        p.nprim = c->shells[sa].nprim * c->shells[sb].nprim;
        for (int k = 0; k < p.nprim; ++k) c->prim_owner.push_back((int)c->pairs.size());
        c->nprim_pairs += p.nprim;
        const int pc = pclass(c->shells[sa].l, c->shells[sb].l);
        c->pairs_by_class[pc].push_back((int)c->pairs.size());
        c->pair_class.push_back(pc);
        c->pairs.push_back(p);
      }
  }
}

// Host threads for the work lists: OMP_NUM_THREADS when set (the CPU share
// the process is meant to use), else the hardware's, at most 16.
int host_threads() {
  int n = (int)std::thread::hardware_concurrency();
  if (const char* v = std::getenv("OMP_NUM_THREADS")) {
    const int e = std::atoi(v);
    if (e > 0) n = e;
  }
  return std::max(1, std::min(16, n));
}

// Work lists for the Fock build (see file comment).
// Host part of the work lists (no HIP calls, no device buffers): it may run
// on a worker thread while the context's stream computes something else.
void build_work_host(bscf_ctx* c, double tau, double split) {
  const double t_start = now_ms();
  const int NPC = kNumPairClasses;
  // host threads over ntasks independent tasks (errors rethrown here)
  auto run_tasks = [&](int ntasks, auto&& task) {
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> err(ntasks);
    auto worker = [&] {
      for (int t; (t = next++) < ntasks;) {
        try {
          task(t);
        } catch (...) {
          err[t] = std::current_exception();
        }
      }
    };
    const int nth = host_threads();
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
  };

  // per instance, per pair class: subclasses keyed by primitive count
  struct Sub {
    int nprim;
    std::vector<int> ids;   // sorted by Q desc
    std::vector<double> q;
    int ket_off;
  };
  std::vector<std::vector<std::vector<Sub>>> subs(c->ninst, std::vector<std::vector<Sub>>(NPC));
  std::vector<int> sub_of(c->pairs.size()), rank_of(c->pairs.size());
  for (int pc = 0; pc < NPC; ++pc)
    for (int pid : c->pairs_by_class[pc]) {
      const int inst = c->shells[c->pairs[pid].a].inst;
      auto& v = subs[inst][pc];
      int k = 0;
      while (k < (int)v.size() && v[k].nprim != c->pairs[pid].nprim) ++k;
      if (k == (int)v.size()) v.push_back(Sub{c->pairs[pid].nprim, {}, {}, 0});
      v[k].ids.push_back(pid);
    }
  // every subclass's kets in descending Schwarz bound (instances in parallel)
  run_tasks(c->ninst, [&](int i) {
    for (int pc = 0; pc < NPC; ++pc) {
      auto& v = subs[i][pc];
      std::sort(v.begin(), v.end(), [](const Sub& x, const Sub& y) { return x.nprim > y.nprim; });
      for (auto& sb : v) {
        std::stable_sort(sb.ids.begin(), sb.ids.end(),
                         [&](int x, int y) { return c->Q[x] > c->Q[y]; });
        sb.q.resize(sb.ids.size());
        for (size_t r = 0; r < sb.ids.size(); ++r) sb.q[r] = c->Q[sb.ids[r]];
      }
    }
  });
  c->kets.clear();
  for (int i = 0; i < c->ninst; ++i)
    for (int pc = 0; pc < NPC; ++pc) {
      auto& v = subs[i][pc];
      for (int s = 0; s < (int)v.size(); ++s) {
        auto& sb = v[s];
        sb.ket_off = (int)c->kets.size();
        for (size_t r = 0; r < sb.ids.size(); ++r) {
          sub_of[sb.ids[r]] = s;
          rank_of[sb.ids[r]] = (int)r;
          c->kets.push_back(sb.ids[r]);
        }
      }
    }
  {
    std::vector<int2> kpos(c->kets.size());
    std::vector<int> kmap;
    c->max_prims = 1;
    std::fill(c->max_prims_pc, c->max_prims_pc + kNumPairClasses, 1);
    for (int i = 0; i < c->ninst; ++i)
      for (int pc = 0; pc < NPC; ++pc)
        for (const Sub& sb : subs[i][pc]) {
          const int ns = (int)sb.ids.size(), kp0 = (int)kmap.size();
          kmap.resize(kp0 + (size_t)ns * sb.nprim);
          for (int r = 0; r < ns; ++r) {
            const ShellPair& pr = c->pairs[sb.ids[r]];
            kpos[sb.ket_off + r] = make_int2(kp0 + r, ns);
            for (int j = 0; j < pr.nprim; ++j) kmap[kp0 + (size_t)j * ns + r] = pr.prim0 + j;
          }
          c->max_prims = std::max(c->max_prims, sb.nprim);
          c->max_prims_pc[pc] = std::max(c->max_prims_pc[pc], sb.nprim);
        }
    c->h_kpos.swap(kpos);
    c->h_kmap.swap(kmap);
  }
  const QuartetClass* qc = quartet_classes();
  struct Tmp {
    WorkItem w;
    double cost;
    int inst;   // instance of the rows
  };
  // The lists of one (class, instance), row indices local to the part; the
  // class's lists are the parts in instance order.
  struct Part {
    std::vector<WorkRow> rows;     // item rows (grouped by primitive counts)
    std::vector<Tmp> tmp;          // 64-quartet items over them
    std::vector<WorkRow> urows;
    std::vector<Tmp> utmp;         // per-bra units over urows
    double nquart = 0, nprimq = 0, nquart32 = 0;
  };
  const int ni = c->ninst;
  std::vector<Part> parts((size_t)kNumQuartetClasses * ni);
  // count of kets of a Q-descending list with qb * q >= thr
  auto prefix = [](const std::vector<double>& q, double qb, double thr) {
    int lo = 0, hi = (int)q.size();
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (qb * q[mid] >= thr) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  // A class whose tuned Fock kernels (every precision tuned so far) and
  // gradient kernel are lane forms never launches a cooperative kernel in
  // this context, so its 64-quartet items (the bulk of the merge for the
  // light classes) are not built; tuning a further precision first rebuilds
  // the lists with every class's items (items_all).
  std::vector<char> skip_items(kNumQuartetClasses, 0);
  if (!c->items_all && c->grad_tuned && (c->fock_tuned[0] || c->fock_tuned[1]))
    for (int q = 0; q < kNumQuartetClasses; ++q)
      skip_items[q] = c->grad_variant[q] == 0 &&
                      (!c->fock_tuned[0] || c->fock_variant[0][q] != 1) &&
                      (!c->fock_tuned[1] || c->fock_variant[1][q] != 1);
  auto build_part = [&](int q, int i) {
    Part& P = parts[(size_t)q * ni + i];
    const int X = pclass(qc[q].la, qc[q].lb), Y = pclass(qc[q].lc, qc[q].ld);
    // units of one bra over its unit rows [r0, r1): up to unit_quartets()
    // consecutive quartets across its rows (all ket primitive counts)
    const int kUnitQuartets = unit_quartets(c->max_n);
    auto add_units = [&](int r0, const std::vector<int>& kn, int bnprim) {
      auto& rows = P.urows;
      const int r1 = (int)rows.size();
      int rr = r0, off = 0;
      while (rr < r1) {
        WorkItem u{rr, off, 0, 0};
        double cost = 0.0;
        while (u.count < kUnitQuartets && rr < r1) {
          const int t = std::min(rows[rr].nket - off, kUnitQuartets - u.count);
          u.count += t;
          cost += double(t) * bnprim * kn[rr - r0];
          off += t;
          if (off == rows[rr].nket) {
            ++rr;
            off = 0;
          }
        }
        P.utmp.push_back({u, cost, i});
      }
    };
    std::vector<int> ur_nprim;
    // rows of this instance grouped by (bra, ket) primitive counts
    std::vector<std::pair<std::pair<int, int>, std::vector<WorkRow>>> groups;
    for (const Sub& bs : subs[i][X])
      for (size_t r = 0; r < bs.ids.size(); ++r) {
        const int bra = bs.ids[r];
        const double qb = bs.q[r];
        const int sb = sub_of[bra];
        const auto& kv = subs[i][Y];
        const int ur0 = (int)P.urows.size();
        ur_nprim.clear();
        for (int t = 0; t < (int)kv.size(); ++t) {
          const Sub& ks = kv[t];
          int lim = tau > 0.0 ? prefix(ks.q, qb, tau) : (int)ks.q.size();
          if (X == Y) {
            if (t > sb) lim = 0;
            else if (t == sb) lim = std::min(lim, (int)r + 1);
          }
          if (lim == 0) continue;
          const int n64 = std::min(lim, prefix(ks.q, qb, split));
          const std::pair<int, int> key(bs.nprim, ks.nprim);
          size_t g = 0;
          while (g < groups.size() && groups[g].first != key) ++g;
          if (g == groups.size()) groups.push_back({key, {}});
          groups[g].second.push_back(WorkRow{bra, ks.ket_off, lim, 0});
          P.urows.push_back(WorkRow{bra, ks.ket_off, lim, n64});   // pad: FP64 prefix
          ur_nprim.push_back(ks.nprim);
          P.nquart32 += lim - n64;
          P.nquart += lim;
          P.nprimq += double(lim) * bs.nprim * ks.nprim;
        }
        add_units(ur0, ur_nprim, bs.nprim);
      }
    // tile every group with items of up to 64 quartets (one per lane)
    if (skip_items[q]) return;
    for (auto& gr : groups) {
      const int r0 = (int)P.rows.size();
      P.rows.insert(P.rows.end(), gr.second.begin(), gr.second.end());
      const int r1 = (int)P.rows.size();
      const double cost = double(gr.first.first) * gr.first.second;
      int r = r0, off = 0;
      while (r < r1) {
        WorkItem w{r, off, 0, 0};
        while (w.count < kWave && r < r1) {
          const int t = std::min(P.rows[r].nket - off, kWave - w.count);
          w.count += t;
          off += t;
          if (off == P.rows[r].nket) {
            ++r;
            off = 0;
          }
        }
        P.tmp.push_back({w, cost, i});
      }
    }
  };
  auto merge_class = [&](int q) {
    auto& W = c->work[q];
    W.nquart = W.nprimq = W.nquart32 = 0;
    W.inst_quart.assign(ni, 0.0);
    W.inst_primq.assign(ni, 0.0);
    W.inst_quart32.assign(ni, 0.0);
    std::vector<Tmp> tmp, utmp;
    W.rows.clear();
    W.ul.rows.clear();
    {
      size_t nr = 0, nt = 0, nur = 0, nut = 0;
      for (int i = 0; i < ni; ++i) {
        const Part& P = parts[(size_t)q * ni + i];
        nr += P.rows.size();
        nt += P.tmp.size();
        nur += P.urows.size();
        nut += P.utmp.size();
      }
      W.rows.reserve(nr);
      tmp.reserve(nt);
      W.ul.rows.reserve(nur);
      utmp.reserve(nut);
    }
    for (int i = 0; i < ni; ++i) {
      Part& P = parts[(size_t)q * ni + i];
      const int r0 = (int)W.rows.size();
      W.rows.insert(W.rows.end(), P.rows.begin(), P.rows.end());
      for (Tmp t : P.tmp) {
        t.w.row += r0;
        tmp.push_back(t);
      }
      const int u0 = (int)W.ul.rows.size();
      W.ul.rows.insert(W.ul.rows.end(), P.urows.begin(), P.urows.end());
      for (Tmp t : P.utmp) {
        t.w.row += u0;
        utmp.push_back(t);
      }
      W.nquart += P.nquart;
      W.nprimq += P.nprimq;
      W.nquart32 += P.nquart32;
      W.inst_quart[i] = P.nquart;
      W.inst_primq[i] = P.nprimq;
      W.inst_quart32[i] = P.nquart32;
      P = Part();   // release the part
    }
    // most expensive first, by counting sorts (stable).  An item's cost is
    // the product of its bra and ket primitive counts, an integer: exact
    // order.  A unit's cost is a sum over its rows; units are ordered by
    // eighths of an octave of it (the order only schedules the work).
    // Items and units go most expensive first.  With kXcds or more instances
    // they are then dealt so that the one at launch position L belongs to an
    // instance i with i % kXcds == L % kXcds: the dispatcher deals workgroups
    // to the XCDs in turn, so each XCD works on its own instances and keeps
    // their ket data in its L2 (a cooperative launch runs the 64 quartets of
    // the item at position p on XCD p % kXcds).  Each XCD's share stays in
    // cost order; once one XCD's share runs out, the rest follow in cost
    // order.  Both orders are counting sorts (stable).
    auto deal = [&](const std::vector<Tmp>& v, std::vector<WorkItem>& out, auto&& key, int nk) {
      const int nx = ni >= kXcds ? kXcds : 1;
      auto xkey = [&](const Tmp& t) { return (nx > 1 ? t.inst % kXcds : 0) * nk + key(t.cost); };
      // one counting sort by (XCD, cost key): XCD x's share, in cost order,
      // ends up in sorted[begin[x], begin[x + 1])
      std::vector<int> start(nx * nk + 1, 0);
      for (const Tmp& t : v) ++start[xkey(t) + 1];
      for (int b = 0; b < nx * nk; ++b) start[b + 1] += start[b];
      std::vector<int> begin(nx + 1);
      for (int x = 0; x <= nx; ++x) begin[x] = start[x * nk];
      std::vector<WorkItem> sorted(v.size());
      std::vector<int> skey(nx > 1 ? v.size() : 0);
      for (const Tmp& t : v) {
        const int k = xkey(t), pos = start[k]++;
        sorted[pos] = t.w;
        if (nx > 1) skey[pos] = k % nk;
      }
      if (nx == 1) {
        out.swap(sorted);
        return;
      }
      out.clear();
      out.reserve(sorted.size());
      int take = begin[1] - begin[0];
      for (int x = 1; x < nx; ++x) take = std::min(take, begin[x + 1] - begin[x]);
      for (int r = 0; r < take; ++r)
        for (int x = 0; x < nx; ++x) out.push_back(sorted[begin[x] + r]);
      // the rest by cost key (a counting sort over what is left)
      std::vector<int> rs(nk + 1, 0);
      for (int x = 0; x < nx; ++x)
        for (int p = begin[x] + take; p < begin[x + 1]; ++p) ++rs[skey[p] + 1];
      for (int b = 0; b < nk; ++b) rs[b + 1] += rs[b];
      const size_t base = out.size();
      out.resize(sorted.size());
      for (int x = 0; x < nx; ++x)
        for (int p = begin[x] + take; p < begin[x + 1]; ++p) out[base + rs[skey[p]]++] = sorted[p];
    };
    // item keys: 4096 - cost (primitive counts per shell pair stay below 64);
    // unit keys: 320 - eighths of octaves (costs stay below 2^40)
    deal(tmp, W.items, [](double cst) { return 4096 - std::min((int)cst, 4096); }, 4097);
    deal(utmp, W.ul.units, [](double cst) {
      const int b = cst > 1.0 ? (int)(8.0 * std::log2(cst)) : 0;
      return 320 - std::min(b, 320);
    }, 321);
    W.has_work = W.nquart > 0;
    W.items_skipped = skip_items[q] != 0;
    W.max_prims = c->max_prims_pc[pclass(qc[q].la, qc[q].lb)];
    W.lds_ok = sizeof(double) * (size_t)unit_lds_doubles(qc[q].la, qc[q].lb, c->max_n,
                                                          W.max_prims) <= c->max_lds_bytes;
  };
  // host threads: first every (class, instance) part, then every class's merge
  // parts interleaved over classes, so that the large classes spread over the threads
  const double t_parts = now_ms();
  run_tasks(kNumQuartetClasses * ni, [&](int t) { build_part(t % kNumQuartetClasses, t / kNumQuartetClasses); });
  const double t_merge = now_ms();
  run_tasks(kNumQuartetClasses, [&](int q) { merge_class(q); });
  c->t_work_phase_ms[0] += t_parts - t_start;
  c->t_work_phase_ms[1] += t_merge - t_parts;
  c->t_work_phase_ms[2] += now_ms() - t_merge;
  c->max_ncd = 0;
  for (int pid : c->kets) {
    const ShellPair& pr = c->pairs[pid];
    c->max_ncd = std::max(c->max_ncd, ncart(c->shells[pr.a].l) * ncart(c->shells[pr.b].l));
  }
  c->host_tau = tau;
  c->host_split = split;
  c->t_work_host_ms += now_ms() - t_start;
}

// Device part: uploads, the ket-order primitive copy and the ket-position
// buffers of the lists that build_work_host made.
void build_work_device(bscf_ctx* c) {
  c->drop_fock_graphs();   // they hold the lists' addresses and sizes
  c->d_kpos.upload(c->h_kpos, c->stream);
  c->d_kmap.upload(c->h_kmap, c->stream);
  c->d_kprims.resize(c->h_kmap.size());
  launch_gather_prims((int)c->h_kmap.size(), c->d_kmap.p, c->d_prims.p, c->d_kprims.p, c->stream);
  for (int q = 0; q < kNumQuartetClasses; ++q) {
    auto& W = c->work[q];
    W.d_items.upload(W.items, c->stream);
    W.d_rows.upload(W.rows, c->stream);
    W.ul.d_units.upload(W.ul.units, c->stream);
    W.ul.d_rows.upload(W.ul.rows, c->stream);
    W.ul.d_keep.resize(W.ul.rows.size());
  }
  c->d_kets.upload(c->kets, c->stream);
  // ket-position buffers; Jk is kept zero between builds by jk_finalize
  const size_t nkb = (size_t)c->max_ncd * c->kets.size();
  c->d_Pk.resize(nkb);
  c->d_Jk.resize(nkb);
  HIPCHK(hipMemsetAsync(c->d_Jk.p, 0, sizeof(double) * c->d_Jk.n, c->stream));
  c->work_tau = c->host_tau;
  c->work_split = c->host_split;
}

// Wait for a work-list build started on a worker thread (rethrowing its
// error); every entry point that reads or replaces the lists calls this first.
void join_work(bscf_ctx* c) {
  if (c->work_job.valid()) {
    const double t0 = now_ms();
    c->work_job.get();
    c->t_work_ms += now_ms() - t0;
  }
}

// Lists for (tau, split) on the device: finish the worker's build when it was
// made for these parameters, else build them here.
void ensure_work(bscf_ctx* c, double tau, double split, bool split_matters) {
  join_work(c);
  if (c->work_tau == tau && (!split_matters || c->work_split == split)) return;
  const double t0 = now_ms();
  if (!(c->host_tau == tau && (!split_matters || c->host_split == split)))
    build_work_host(c, tau, split);
  build_work_device(c);
  c->t_work_ms += now_ms() - t0;
}

// Add the work that incremental builds kept (counted on the device) to the
// statistics and clear the device counts.
void collect_kept(bscf_ctx* c) {
  if (c->d_kept.n == 0) return;
  std::vector<double> h(c->d_kept.n);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_kept.p, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  sync(c);
  const int ni = c->ninst;
  for (int q = 0; q < kNumQuartetClasses; ++q)
    for (int i = 0; i < ni; ++i) {
      c->work[q].done_quart += h[(size_t)q * ni + i];
      c->work[q].done_primq += h[(size_t)(kNumQuartetClasses + q) * ni + i];
      c->work[q].done_quart32 += h[(size_t)(2 * kNumQuartetClasses + q) * ni + i];
    }
  launch_fill(c->d_kept.p, (long long)c->d_kept.n, 0.0, c->stream);
}

// Start a profiled interval on stream s (returns its index) / end it.
int prof_begin(bscf_ctx* c, int q, int kind, hipStream_t s) {
  bscf_ctx::ProfRec r{nullptr, nullptr, q, kind};
  for (hipEvent_t* e : {&r.e0, &r.e1}) {
    if (c->prof_free.empty()) {
      HIPCHK(hipEventCreate(e));
    } else {
      *e = c->prof_free.back();
      c->prof_free.pop_back();
    }
  }
  HIPCHK(hipEventRecord(r.e0, s));
  c->prof_pending.push_back(r);
  return (int)c->prof_pending.size() - 1;
}

void prof_end(bscf_ctx* c, int idx, hipStream_t s) {
  HIPCHK(hipEventRecord(c->prof_pending[idx].e1, s));
}

// Read back every pending interval into the statistics.
void prof_collect(bscf_ctx* c) {
  for (auto& r : c->prof_pending) {
    HIPCHK(hipEventSynchronize(r.e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
    if (r.kind == 0) c->work[r.q].kernel_ms += ms;
    else if (r.kind == 1) c->work[r.q].grad_ms += ms;
    else if (r.kind == 2) c->t_fock_gpu_ms += ms;
    else c->xc_ms[r.q] += ms;
    c->prof_free.push_back(r.e0);
    c->prof_free.push_back(r.e1);
  }
  c->prof_pending.clear();
}

FockArgs fock_args(bscf_ctx* c, double* J, double* K, const int* active) {
  FockArgs a;
  a.items = nullptr;
  a.nitems = 0;
  a.rows = nullptr;
  a.units = nullptr;
  a.nunits = 0;
  a.urows = nullptr;
  a.pairs = c->d_pairs.p;
  a.prims = c->d_prims.p;
  a.shells = c->d_shells.p;
  a.kets = c->d_kets.p;
  a.kprims = c->d_kprims.p;
  a.kpos = c->d_kpos.p;
  a.max_prims = c->max_prims;
  a.moff = c->d_moff.p;
  a.nbf = c->d_nbf.p;
  a.nmax = c->max_n;
  a.nk_total = (int)c->kets.size();
  a.P = c->P.p;
  a.Pk = c->d_Pk.p;
  a.J = J;
  a.Jk = c->d_Jk.p;
  a.K = K;
  a.boys64 = c->d_boys64.p;
  a.boys32 = c->d_boys32.p;
  a.active = active;
  a.ukeep = nullptr;
  a.Q = c->d_Q.p;
  a.dpmax = nullptr;
  a.tau = 0.0;
  a.dPm = nullptr;
  a.pm_off = c->d_pm_off.p;
  a.shell_off = c->d_shell_off.p;
  a.nsh = c->d_nshell.p;
  a.kept_q = a.kept_pq = a.kept_32 = nullptr;
  a.Jfx = a.Kfx = a.Jkfx = nullptr;
  a.unit_threads = 64;
  return a;
}

// Point a at the 64-quartet items and the units of class W.
void set_class(FockArgs& a, const bscf_ctx::ClassWork& W) {
  a.items = W.d_items.p;
  a.nitems = (int)W.items.size();
  a.rows = W.d_rows.p;
  a.units = W.ul.d_units.p;
  a.nunits = (int)W.ul.units.size();
  a.urows = W.ul.d_rows.p;
  a.ukeep = W.ul.d_keep.p;
  a.max_prims = W.max_prims;
}

// Lane-kernel launch of class q: mode 0 every quartet in FP64, mode 2 the
// quartets above the split in FP64 and the rest in FP32, in one launch.
template <class Launch>
void lane_launches(bscf_ctx* c, FockArgs& a, int q, int mode, Launch&& launch) {
  const QuartetClass* qc = quartet_classes();
  const auto& W = c->work[q];
  set_class(a, W);
  if (mode == 2) launch(1, [&](hipStream_t s) { qc[q].fock(a, 2, s); });
  else launch(0, [&](hipStream_t s) { qc[q].fock(a, 0, s); });
}

// lane mode of class q under the chosen variant
int lane_mode(bscf_ctx* c, int precision, int q) {
  return (precision == BSCF_MIXED && c->fock_variant[1][q] == 0) ? 2 : 0;
}

KetPosArgs ketpos_args(bscf_ctx* c) {
  KetPosArgs k;
  k.nk_total = (int)c->kets.size();
  k.kets = c->d_kets.p;
  k.pairs = c->d_pairs.p;
  k.shells = c->d_shells.p;
  k.moff = c->d_moff.p;
  k.nbf = c->d_nbf.p;
  return k;
}

// Time the lane and cooperative kernels of every class that has both on the
// current work lists (second of two runs each, into throwaway J and K) and keep
// the faster; BSCF_VARIANT=lane|coop forces a choice.  A class whose lane
// kernel needs more LDS than one workgroup may hold runs cooperatively.
void autotune_fock(bscf_ctx* c, int pcol) {
  c->drop_fock_graphs();   // they hold the tuned kernels and launch shapes
  const char* env = getenv("BSCF_VARIANT");
  // BSCF_UNIT_THREADS=64|128|256 fixes the threads of the lane units
  const char* env_u = getenv("BSCF_UNIT_THREADS");
  const int env_nt = env_u ? atoi(env_u) : 0;
  need(env_nt == 0 || env_nt == 64 || env_nt == 128 || env_nt == 256, BSCF_E_INVALID,
       "BSCF_UNIT_THREADS must be 64, 128 or 256");
  const QuartetClass* qc = quartet_classes();
  FockArgs a = fock_args(c, c->tmp1.p, c->tmp2.p, c->d_all_active.p);
  const KetPosArgs kp = ketpos_args(c);
  launch_gather_pk(kp, c->max_ncd, c->P.p, c->d_Pk.p, c->stream);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int q = 0; q < kNumQuartetClasses; ++q) {
    auto& W = c->work[q];
    for (float& t : c->tune_ms[pcol][q]) t = 0.0f;
    const bool lane_ok = qc[q].fock && W.lds_ok && c->private_bytes[q][0] <= c->lane_scratch_max &&
                         !(pcol && c->private_bytes[q][1] > c->lane_scratch_max);
    if (!lane_ok) c->fock_variant[pcol][q] = 1;
    if (!W.has_work) continue;
    set_class(a, W);
    // variants: 0 the lane form of this precision, 1 cooperative, and in
    // MIXED mode 2 the FP64 lane form (FP32 integrals do not pay everywhere);
    // each timed alone (second of two runs), the chosen one at least, since
    // the build's stream schedule uses its time
    // lane forms also try units of one, two and four wavefronts (they share
    // the unit's LDS rows) and keep the fastest
    auto time_variant = [&](int v) {
      float best = -1.0f;
      c->unit_threads[pcol][q][v] = 64;
      for (int nt : {64, 128, 256}) {
        if (v == 1 && nt != 64) break;
        if (env_nt > 0 && v != 1 && nt != env_nt) continue;
        a.unit_threads = nt;
        for (int rep = 0; rep < 2; ++rep) {
          HIPCHK(hipEventRecord(e0, c->stream));
          if (v == 1) qc[q].coop_fock(a, c->stream);
          else lane_launches(c, a, q, (pcol && v == 0) ? 2 : 0,
                             [&](int, auto&& run) { run(c->stream); });
          HIPCHK(hipEventRecord(e1, c->stream));
        }
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (best < 0.0f || ms < best) {
          best = ms;
          if (v != 1) c->unit_threads[pcol][q][v] = nt;
        }
      }
      c->tune_ms[pcol][q][v] = best;
      a.unit_threads = 64;
    };
    int forced = -1;
    if (!lane_ok) forced = 1;
    else if (env && !strcmp(env, "lane")) forced = 0;
    else if (env && !strcmp(env, "coop")) forced = 1;
    if (forced >= 0) {
      c->fock_variant[pcol][q] = forced;
      time_variant(forced);
      continue;
    }
    const int nv = pcol ? 3 : 2;
    for (int v = 0; v < nv; ++v) time_variant(v);
    int best = 0;
    for (int v = 1; v < nv; ++v)
      if (c->tune_ms[pcol][q][v] < c->tune_ms[pcol][q][best]) best = v;
    c->fock_variant[pcol][q] = best;
  }
  // the lane runs left ket-side sums in Jk: fold them into the throwaway J
  launch_jk_finalize(kp, c->max_ncd, c->d_Jk.p, c->tmp1.p, c->stream);
  HIPCHK(hipGetLastError());
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->fock_tuned[pcol] = true;
}

// One Fock build.  Full: J and K from P over every listed quartet.
// Incremental (Almlof's direct SCF): J and K keep the last build's values and
// gain the contributions of dP = P - Pprev, from the quartets with
// Q_ab Q_cd min(max|dP|, 1) >= tau; J and K are linear in the density, so
// only the skipped quartets (each bounded by tau) differ from a full build.
// ------------------------------------------------------------------ B3LYP

// Chunk buffers hold at most this many doubles each (2 GiB): a run of
// instances takes its grid points in chunks of G = budget / (count n),
// a multiple of the slice width kXcSlice
constexpr size_t kXcBudget = size_t(1) << 28;
// V += X^T B reduces over the chunk's points; the library GEMM is slow for a
// reduction dimension far above n, so the chunk is cut into slices of this
// many points, one batched GEMM covers every (instance, slice) and a kernel
// sums the slices in order
constexpr int kXcSlice = 8192;
// steps of an XC build as timed by the statistics
// steps of the XC build, then the XC gradient's basis-function and weight terms
enum XcStep { kXcBasis = 0, kXcGemm = 1, kXcPoint = 2, kXcGemmV = 3, kXcWhole = 4, kXcGradOrb = 5,
              kXcGradWeight = 6 };

// Radial and angular tables of the grid (xc.h), once per context
void xc_tables(bscf_ctx* c) {
  auto& x = c->xcs;
  if (x.tables) return;
  std::vector<double> rr(2 * kXcRad), rw(2 * kXcRad);
  for (int t = 0; t < 2; ++t) {
    const double R = t == 0 ? 1.0 : 0.6;
    for (int i = 1; i <= kXcRad; ++i) {
      const double th = i * M_PI / (kXcRad + 1), xx = std::cos(th);
      const double r = R * (1 + xx) / (1 - xx);
      const double w = M_PI / (kXcRad + 1) * std::sin(th) * std::sin(th);
      rr[t * kXcRad + i - 1] = r;
      rw[t * kXcRad + i - 1] = w * r * r * (2 * R / ((1 - xx) * (1 - xx))) / std::sqrt(1 - xx * xx);
    }
  }
  // Gauss-Legendre nodes in cos(theta) by Newton's method on P_n
  std::vector<double> ct(kXcTheta), wt(kXcTheta);
  for (int k = 0; k < kXcTheta; ++k) {
    double z = std::cos(M_PI * (k + 0.75) / (kXcTheta + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int m = 2; m <= kXcTheta; ++m) {
        const double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = kXcTheta * (z * p1 - p0) / (z * z - 1);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    ct[k] = z;
    wt[k] = 2.0 / ((1 - z * z) * dp * dp);
  }
  std::vector<double> au(3 * kXcAng), aw(kXcAng);
  const int nphi = 2 * kXcTheta;
  for (int k = 0; k < kXcTheta; ++k)
    for (int m = 0; m < nphi; ++m) {
      const int j = k * nphi + m;
      const double st = std::sqrt(1 - ct[k] * ct[k]), ph = 2 * M_PI * m / nphi;
      au[3 * j] = st * std::cos(ph);
      au[3 * j + 1] = st * std::sin(ph);
      au[3 * j + 2] = ct[k];
      aw[j] = wt[k] * 2 * M_PI / nphi;
    }
  x.h_rad_r = rr;
  x.h_ang_u = au;
  // sectors: cos(theta) >= 0 or < 0 (the first or last kXcTheta / 2 nodes,
  // in decreasing cos(theta)) times sin(phi) >= 0 or < 0 (phi below or from pi)
  std::vector<int> sec(kXcAng);
  {
    int fill[kXcSectors] = {};
    for (int k = 0; k < kXcTheta; ++k)
      for (int m = 0; m < nphi; ++m) {
        const int sc = (k >= kXcTheta / 2 ? 2 : 0) + (m >= nphi / 2 ? 1 : 0);
        sec[sc * kXcSectorAng + fill[sc]++] = k * nphi + m;
      }
  }
  x.d_sec_ang.upload(sec, c->stream);
  x.rad_r.upload(rr, c->stream);
  x.rad_w.upload(rw, c->stream);
  x.ang_u.upload(au, c->stream);
  x.ang_w.upload(aw, c->stream);
  x.tables = true;
}

// Sparse chunks of every group whose instances have the same atoms: per atom,
// block of kXcSparseShells radial shells (points at distances r_lo..r_hi from
// the atom) and angular sector, the basis shells whose values or gradients can
// exceed kXcShellEps there in some instance of the group.  Bound at a lower
// bound d of the distance from the shell's centre to the chunk's points:
// sum_k |c_k| exp(-a_k d^2) (d + 3)^l (1 + 2 a_k (d + 3)).  With v the shell
// centre relative to the atom, D = |v| and c >= the largest u . v / D over
// the sector's directions u, every point r u of the chunk has |r u - v|^2 >=
// r^2 - 2 r D c + D^2, least at r = clamp(D c, r_lo, r_hi).  A sector is the
// convex cone s_z u_z >= 0, s_y u_y >= 0, so c = |(v_x, max(s_y v_y, 0),
// max(s_z v_z, 0))| / D (the norm of v's projection onto the cone).
void xc_chunks(bscf_ctx* c) {
  auto& x = c->xcs;
  x.gch.assign(c->groups.size(), {});
  std::vector<int> shl, scbf, fmap, meta;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& gr = c->groups[gi];
    auto& G = x.gch[gi];
    const int i0 = gr.first, na = c->natoms[i0];
    bool same = true;
    for (int i = i0 + 1; i < gr.first + gr.count && same; ++i) {
      same = c->natoms[i] == na && c->nshell[i] == c->nshell[i0];
      for (int a = 0; a < na && same; ++a) same = c->Zs[c->atom_off[i] + a] == c->Zs[c->atom_off[i0] + a];
    }
    if (!same) continue;
    G.sparse = true;
    const int nsh = c->nshell[i0];
    // per shell the distance beyond which the bound stays below kXcShellEps:
    // the bound, a sum of e^{-a d^2} times polynomials in d, decreases past
    // its maxima (at d of a bohr or two), far before it reaches 1e-14, so the
    // last point of a 0.05-bohr scan where it is still above, plus one step
    std::vector<double> rcut(nsh, 0.0);
    for (int s = 0; s < nsh; ++s) {
      const Shell& sh = c->shells[c->shell_off[i0] + s];
      auto bound = [&](double d) {
        const double dp = d + 3.0;
        double b = 0.0;
        for (int k = 0; k < sh.nprim; ++k) {
          const double al = c->sh_exp[sh.prim0 + k];
          b += std::fabs(c->sh_coef[sh.prim0 + k]) * std::exp(-al * d * d) * (1.0 + 2.0 * al * dp);
        }
        return b * std::pow(dp, sh.l);
      };
      double last = -1.0;
      for (double d = 0.0; d < 400.0; d += 0.05) {
        const double b = bound(d);
        if (b > kXcShellEps) last = d;
        else if (last >= 0.0 && b < 1e-6 * kXcShellEps) break;
      }
      rcut[s] = last < 0.0 ? -1.0 : last + 0.05;
    }
    for (int a = 0; a < na; ++a) {
      const int tab = c->Zs[c->atom_off[i0] + a] == 1 ? 0 : 1;
      for (int r0 = 0; r0 < kXcRad; r0 += kXcSparseShells)
      for (int sc = 0; sc < kXcSectors; ++sc) {
        const int r1 = std::min(kXcRad, r0 + kXcSparseShells);
        const double sy = (sc & 1) ? -1.0 : 1.0, sz = (sc & 2) ? -1.0 : 1.0;
        double rlo = 1e300, rhi = 0.0;
        for (int r = r0; r < r1; ++r) {
          rlo = std::min(rlo, x.h_rad_r[tab * kXcRad + r]);
          rhi = std::max(rhi, x.h_rad_r[tab * kXcRad + r]);
        }
        bscf_ctx::Xcs::Chunk ch;
        ch.p0 = a * kXcPerAtom + r0 * kXcAng;
        ch.gcnt = (r1 - r0) * kXcSectorAng;
        ch.sh0 = (int)shl.size();
        ch.f0 = (int)fmap.size();
        ch.sec = sc;
        int nf = 0;
        for (int s = 0; s < nsh; ++s) {
          bool keep = false;
          for (int i = i0; i < gr.first + gr.count && !keep; ++i) {
            const Shell& sh = c->shells[c->shell_off[i] + s];
            const double* A = &c->xyz[3 * (size_t)(c->atom_off[i] + a)];
            const double vx = sh.x - A[0], vy = sh.y - A[1], vz = sh.z - A[2];
            const double d = std::sqrt(vx * vx + vy * vy + vz * vz);
            double dm = rlo;   // the shell sits on the atom
            if (d > 0.0) {
              const double py = std::max(sy * vy, 0.0), pz = std::max(sz * vz, 0.0);
              const double cmax = std::min(1.0, std::sqrt(vx * vx + py * py + pz * pz) / d);
              const double rs = std::min(rhi, std::max(rlo, d * cmax));
              dm = std::sqrt(std::max(0.0, rs * rs - 2.0 * rs * d * cmax + d * d));
            }
            keep = dm <= rcut[s];
          }
          if (!keep) continue;
          const Shell& sh = c->shells[c->shell_off[i0] + s];
          shl.push_back(s);
          scbf.push_back(nf);
          for (int k = 0; k < ncart(sh.l); ++k) fmap.push_back(sh.bf + k);
          nf += ncart(sh.l);
        }
        ch.nsh = (int)shl.size() - ch.sh0;
        ch.ns = nf;
        if (nf > 0) G.chunks.push_back(ch);
      }
    }
    // largest first; a bucket takes the chunks whose width padded to a
    // multiple of 16 is at least 70% of its first one's (so the narrowest
    // chunks, all padded to 16, share one bucket)
    std::stable_sort(G.chunks.begin(), G.chunks.end(),
                     [](const bscf_ctx::Xcs::Chunk& p, const bscf_ctx::Xcs::Chunk& q) { return p.ns > q.ns; });
    for (int k = 0; k < (int)G.chunks.size();) {
      bscf_ctx::Xcs::Bucket b;
      b.c0 = k;
      b.W = (G.chunks[k].ns + 15) / 16 * 16;
      b.max_nsh = 0;
      do {   // the first chunk always, then those down to 70% of the width
        b.max_nsh = std::max(b.max_nsh, G.chunks[k].nsh);
        ++k;
      } while (k < (int)G.chunks.size() && (G.chunks[k].ns + 15) / 16 * 16 * 10 >= b.W * 7);
      b.nch = k - b.c0;
      G.buckets.push_back(b);
    }
    G.meta0 = (int)meta.size() / kXcMeta;
    for (const auto& ch : G.chunks)
      for (int v : {ch.p0, ch.gcnt, ch.sh0, ch.nsh, ch.f0, ch.ns, ch.sec}) meta.push_back(v);
  }
  x.d_meta.upload(meta, c->stream);
  x.d_shl.upload(shl, c->stream);
  x.d_scbf.upload(scbf, c->stream);
  x.d_fmap.upload(fmap, c->stream);
}

// the molecular grid of every instance at the current geometry
void xc_grid(bscf_ctx* c) {
  auto& x = c->xcs;
  if (x.grid_ok) return;
  xc_tables(c);
  x.pt_off.assign(c->ninst + 1, 0);
  for (int i = 0; i < c->ninst; ++i)
    x.pt_off[i + 1] = x.pt_off[i] + (long long)c->natoms[i] * kXcPerAtom;
  x.npts = x.pt_off[c->ninst];
  x.npts_i.assign(c->ninst, 0);
  for (int i = 0; i < c->ninst; ++i) x.npts_i[i] = (int)(x.pt_off[i + 1] - x.pt_off[i]);
  x.pts.resize((size_t)4 * x.npts);
  x.d_pt_off.upload(x.pt_off, c->stream);
  x.d_npts.upload(x.npts_i, c->stream);
  x.d_sh_off.upload(c->shell_off, c->stream);
  x.d_nsh.upload(c->nshell, c->stream);
  // the grid kernel keeps each point's atom distances in LDS
  need(sizeof(double) * 64 * (size_t)c->max_atoms <= (size_t)c->max_lds_bytes, BSCF_E_UNSUPPORTED,
       "B3LYP grid: too many atoms per instance for the LDS");
  // 1/|R_A - R_B| of every instance's atom pairs (grid weights and their gradient)
  x.isep_off.assign(c->ninst + 1, 0);
  for (int i = 0; i < c->ninst; ++i)
    x.isep_off[i + 1] = x.isep_off[i] + (long long)c->natoms[i] * c->natoms[i];
  std::vector<double> isep(x.isep_off[c->ninst], 0.0);
  for (int i = 0; i < c->ninst; ++i) {
    const int na = c->natoms[i];
    const double* X = &c->xyz[3 * (size_t)c->atom_off[i]];
    for (int A = 0; A < na; ++A)
      for (int B = 0; B < na; ++B)
        if (A != B)
          isep[x.isep_off[i] + (long long)A * na + B] =
              1.0 / std::sqrt((X[3 * A] - X[3 * B]) * (X[3 * A] - X[3 * B]) +
                              (X[3 * A + 1] - X[3 * B + 1]) * (X[3 * A + 1] - X[3 * B + 1]) +
                              (X[3 * A + 2] - X[3 * B + 2]) * (X[3 * A + 2] - X[3 * B + 2]));
  }
  x.isep.upload(isep, c->stream);
  for (int i = 0; i < c->ninst; ++i) {
    XcGridArgs g;
    g.npts = (int)(x.pt_off[i + 1] - x.pt_off[i]);
    g.natoms = c->natoms[i];
    g.xyz = c->d_xyz.p + 3LL * c->atom_off[i];
    g.Z = c->d_Zd.p + c->atom_off[i];
    g.rad_r = x.rad_r.p;
    g.rad_w = x.rad_w.p;
    g.ang_u = x.ang_u.p;
    g.ang_w = x.ang_w.p;
    g.pts = x.pts.p + 4 * x.pt_off[i];
    g.inv_sep = x.isep.p + x.isep_off[i];
    launch_xc_grid(g, c->stream);
  }
  HIPCHK(hipGetLastError());
  xc_chunks(c);
  x.grid_ok = true;
}

// V_xc and E_xc of every (active, if masked) instance at the densities P:
// per run of consecutive active instances of one group (equal basis size),
// batched over the run's instances, in chunks of grid points
void xc_build(bscf_ctx* c, const double* P, bool masked) {
  auto& x = c->xcs;
  xc_grid(c);
  x.V.resize(c->mtot);
  x.exc.resize(c->ninst);
  const hipStream_t st = c->stream;
  const int pw = c->profiling ? prof_begin(c, kXcWhole, 3, st) : -1;
  launch_fill(x.exc.p, c->ninst, 0.0, st);
  // one XC step, bracketed by events when profiling
  auto step = [&](int q, auto&& f) {
    const int pk = c->profiling ? prof_begin(c, q, 3, st) : -1;
    f();
    if (pk >= 0) prof_end(c, pk, st);
    c->xc_launches[q]++;
  };
  const char* dense_env = std::getenv("BSCF_XC_DENSE");   // the dense form everywhere (tests)
  const bool force_dense = dense_env && std::atoi(dense_env) != 0;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& gr = c->groups[gi];
    for (int r0 = gr.first; r0 < gr.first + gr.count;) {
      if (masked && !c->h_active[r0]) {
        ++r0;
        continue;
      }
      int r1 = r0;
      while (r1 < gr.first + gr.count && (!masked || c->h_active[r1])) ++r1;
      const int count = r1 - r0, n = gr.n;
      const auto& GC = x.gch[gi];
      if (GC.sparse && !force_dense) {
        // sparse form: per bucket of chunks, all its chunks times the run's
        // instances in one launch of each step (xc.h)
        const int G = kXcSparseG;
        double* V = x.V.p + c->moff[r0];
        launch_fill(V, (long long)count * n * n, 0.0, st);
        XcSparseArgs a;
        a.G = G;
        a.count = count;
        a.first = r0;
        a.n = n;
        a.sh_list = x.d_shl.p;
        a.sec_ang = x.d_sec_ang.p;
        a.sh_cbf = x.d_scbf.p;
        a.fmap = x.d_fmap.p;
        a.sh_off = x.d_sh_off.p;
        a.shells = c->d_shells.p;
        a.sh_exp = c->d_sh_exp.p;
        a.sh_coef = c->d_sh_coef.p;
        a.pt_off = x.d_pt_off.p;
        a.pts = x.pts.p;
        a.moff = c->d_moff.p;
        a.P = P;
        a.V = x.V.p;
        const double one = 1.0, zero = 0.0;
        for (const auto& bk : GC.buckets) {
          const int W = bk.W;
          // launches of at most the buffer budget
          const int per = std::max<int>(1, (int)(kXcBudget / ((size_t)count * W * G)));
          for (int c0 = 0; c0 < bk.nch; c0 += per) {
            const int nch = std::min(per, bk.nch - c0), slots = nch * count;
            x.B.resize((size_t)slots * W * G);
            x.Z.resize((size_t)slots * W * G);
            x.Ps.resize((size_t)slots * W * W);
            x.Vs.resize((size_t)slots * W * W);
            x.part.resize((size_t)slots * (G / kXcSB));
            a.W = W;
            a.nch = nch;
            a.meta = x.d_meta.p + kXcMeta * (GC.meta0 + bk.c0 + c0);
            a.B = x.B.p;
            a.Z = x.Z.p;
            a.Ps = x.Ps.p;
            a.Vs = x.Vs.p;
            a.part = x.part.p;
            const long long sBZ = (long long)W * G, sP = (long long)W * W;
            step(kXcBasis, [&] {
              launch_xc_sparse_basis(a, bk.max_nsh, st);
              launch_xc_sparse_gather(a, st);
            });
            // Z = B Ps (column-major G x W times W x W, every slot)
            step(kXcGemm, [&] {
              BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                                    rocblas_operation_none, G, W, W, &one, x.B.p,
                                                    G, sBZ, x.Ps.p, W, sP, &zero, x.Z.p, G, sBZ,
                                                    slots));
            });
            step(kXcPoint, [&] {
              launch_xc_sparse_point(a, st);   // Z <- X
              launch_xc_sparse_reduce(a, x.exc.p, st);
            });
            // Vs = X^T B, added into V through the function maps
            step(kXcGemmV, [&] {
              BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose,
                                                    rocblas_operation_none, W, W, G, &one, x.Z.p,
                                                    G, sBZ, x.B.p, G, sBZ, &zero, x.Vs.p, W, sP,
                                                    slots));
              launch_xc_sparse_scatter(a, st);
            });
            c->xc_gemm_flops += 4.0 * G * (double)W * W * slots;
            for (int k = 0; k < nch; ++k) {
              const auto& ch = GC.chunks[bk.c0 + c0 + k];
              c->xc_basis_bytes += (8.0 * ch.ns + 32.0) * ch.gcnt * count;
              c->xc_point_bytes += (16.0 * ch.ns + 32.0) * ch.gcnt * count;
            }
          }
        }
        launch_xc_symmetrize(n, count, V, st);
        for (int i = r0; i < r1; ++i) c->xc_points += x.npts_i[i];
        r0 = r1;
        continue;
      }
      int np_max = 0, nsh_max = 0;
      for (int i = r0; i < r1; ++i) {
        np_max = std::max(np_max, x.npts_i[i]);
        nsh_max = std::max(nsh_max, c->nshell[i]);
      }
      int slice = kXcSlice;
      int cap = (int)std::min<size_t>(kXcBudget / ((size_t)count * n), 1 << 30);
      if (const char* e = std::getenv("BSCF_XC_CHUNK")) {   // chunk width (tests)
        cap = std::min(cap, std::atoi(e));
        slice = std::max(256, std::min(slice, cap / 2 / 256 * 256));
      }
      cap = std::max(slice, cap / slice * slice);
      const int G = std::min((np_max + slice - 1) / slice * slice, cap);
      const int S = G / slice;
      x.B.resize((size_t)count * n * G);
      x.Z.resize((size_t)count * n * G);
      x.part.resize((size_t)count * (G / 256));
      x.Vp.resize((size_t)count * S * n * n);
      x.hgp.resize((size_t)3 * count * S);
      for (int i = 0; i < count; ++i)
        for (int sl = 0; sl < S; ++sl) {
          const size_t k = (size_t)i * S + sl, o = (size_t)i * n * G + (size_t)sl * slice;
          x.hgp[k] = x.Z.p + o;
          x.hgp[(size_t)count * S + k] = x.B.p + o;
          x.hgp[(size_t)2 * count * S + k] = x.Vp.p + k * n * n;
        }
      x.gp.resize(x.hgp.size());
      HIPCHK(hipMemcpyAsync(x.gp.p, x.hgp.data(), x.hgp.size() * sizeof(const double*),
                            hipMemcpyHostToDevice, st));
      XcChunkArgs a;
      a.G = G;
      a.n = n;
      a.first = r0;
      a.npts = x.d_npts.p;
      a.pt_off = x.d_pt_off.p;
      a.sh_off = x.d_sh_off.p;
      a.nsh = x.d_nsh.p;
      a.shells = c->d_shells.p;
      a.sh_exp = c->d_sh_exp.p;
      a.sh_coef = c->d_sh_coef.p;
      a.pts = x.pts.p;
      a.B = x.B.p;
      a.Z = x.Z.p;
      a.part = x.part.p;
      const long long sBZ = (long long)n * G, sP = (long long)n * n;
      double* V = x.V.p + c->moff[r0];
      const double one = 1.0, zero = 0.0;
      for (int g0 = 0; g0 < np_max; g0 += G) {
        a.g0 = g0;
        step(kXcBasis, [&] { launch_xc_basis(a, count, nsh_max, st); });
        // Z = B P: each function-major B is a column-major G x n matrix
        step(kXcGemm, [&] {
          BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                                rocblas_operation_none, G, n, n, &one, x.B.p, G,
                                                sBZ, P + c->moff[r0], n, sP, &zero, x.Z.p, G, sBZ,
                                                count));
        });
        step(kXcPoint, [&] {
          launch_xc_point(a, count, st);   // Z <- X
          launch_xc_reduce(a, count, x.exc.p, st);
        });
        // V (column-major) += X^T B over the chunk: one product per
        // (instance, slice), then their sum; V + V^T at the end (a rank-2k
        // update would do both, but the library's is far slower at k >> n)
        step(kXcGemmV, [&] {
          const double* const* pa = x.gp.p;
          const double* const* pb = x.gp.p + (size_t)count * S;
          BLASCHK(rocblas_dgemm_batched(c->blas, rocblas_operation_transpose,
                                        rocblas_operation_none, n, n, slice, &one, pa, G, pb, G,
                                        &zero, x.gp.p + (size_t)2 * count * S, n, count * S));
          launch_xc_slice_sum(n, count, S, x.Vp.p, V, g0 > 0, st);
        });
        c->xc_gemm_flops += 4.0 * G * (double)n * n * count;
      }
      for (int i = r0; i < r1; ++i) {
        c->xc_points += x.npts_i[i];
        c->xc_basis_bytes += (8.0 * n + 32.0) * x.npts_i[i];
        c->xc_point_bytes += (16.0 * n + 32.0) * x.npts_i[i];
      }
      launch_xc_symmetrize(n, count, V, st);
      r0 = r1;
    }
  }
  if (pw >= 0) prof_end(c, pw, st);
  c->xc_launches[kXcWhole]++;
  c->xc_builds++;
  HIPCHK(hipGetLastError());
}

// dE_xc/dR at the densities P of every instance, added into grad ([total
// atoms][3]): the basis-function term per bucket of the sparse chunks, then
// the Becke-weight term per instance (xc.h).  Needs the sparse form in every
// group (instances of a group with the same atoms).
void xc_gradient(bscf_ctx* c, const double* P, double* grad) {
  auto& x = c->xcs;
  xc_grid(c);
  for (const auto& GC : x.gch)
    need(GC.sparse, BSCF_E_UNSUPPORTED,
         "B3LYP forces need the instances of each basis-size group to have the same atoms");
  // the weight-derivative kernel keeps [natoms][128 + 3] doubles in LDS
  need(sizeof(double) * (128 + 3) * (size_t)c->max_atoms <= (size_t)c->max_lds_bytes,
       BSCF_E_UNSUPPORTED, "B3LYP forces: too many atoms per instance for the LDS");
  const hipStream_t st = c->stream;
  x.eg.resize((size_t)x.npts);
  const int p1 = c->profiling ? prof_begin(c, kXcGradOrb, 3, st) : -1;
  launch_fill(x.eg.p, x.npts, 0.0, st);
  const double one = 1.0, zero = 0.0;
  const int G = kXcSparseG;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& gr = c->groups[gi];
    const auto& GC = x.gch[gi];
    const int count = gr.count, n = gr.n;
    XcSparseArgs a;
    a.G = G;
    a.count = count;
    a.first = gr.first;
    a.n = n;
    a.sh_list = x.d_shl.p;
    a.sec_ang = x.d_sec_ang.p;
    a.sh_cbf = x.d_scbf.p;
    a.fmap = x.d_fmap.p;
    a.sh_off = x.d_sh_off.p;
    a.shells = c->d_shells.p;
    a.sh_exp = c->d_sh_exp.p;
    a.sh_coef = c->d_sh_coef.p;
    a.pt_off = x.d_pt_off.p;
    a.pts = x.pts.p;
    a.moff = c->d_moff.p;
    a.P = P;
    a.V = nullptr;
    for (const auto& bk : GC.buckets) {
      const int W = bk.W;
      const int per = std::max<int>(1, (int)(kXcBudget / ((size_t)count * W * G)));
      for (int c0 = 0; c0 < bk.nch; c0 += per) {
        const int nch = std::min(per, bk.nch - c0), slots = nch * count;
        x.B.resize((size_t)slots * W * G);
        x.Z.resize((size_t)slots * W * G);
        x.Yg.resize((size_t)slots * W * G);
        x.Ps.resize((size_t)slots * W * W);
        x.gf.resize((size_t)slots * 5 * G);
        a.W = W;
        a.nch = nch;
        a.meta = x.d_meta.p + kXcMeta * (GC.meta0 + bk.c0 + c0);
        a.B = x.B.p;
        a.Z = x.Z.p;
        a.Ps = x.Ps.p;
        a.Vs = nullptr;
        a.part = nullptr;
        const long long sBZ = (long long)W * G, sP = (long long)W * W;
        launch_xc_sparse_basis(a, bk.max_nsh, st);
        launch_xc_sparse_gather(a, st);
        // Z = B Ps
        BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                              rocblas_operation_none, G, W, W, &one, x.B.p, G,
                                              sBZ, x.Ps.p, W, sP, &zero, x.Z.p, G, sBZ, slots));
        launch_xc_sparse_gpoint(a, x.gf.p, x.eg.p, st);   // B <- D
        // Y = D Ps
        BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                              rocblas_operation_none, G, W, W, &one, x.B.p, G,
                                              sBZ, x.Ps.p, W, sP, &zero, x.Yg.p, G, sBZ, slots));
        launch_xc_sparse_force(a, bk.max_nsh, x.gf.p, x.Yg.p, c->d_atom_off.p, grad, st);
      }
    }
  }
  if (p1 >= 0) prof_end(c, p1, st);
  c->xc_launches[kXcGradOrb]++;
  const int p2 = c->profiling ? prof_begin(c, kXcGradWeight, 3, st) : -1;
  for (int i = 0; i < c->ninst; ++i) {
    XcGridArgs g;
    g.npts = x.npts_i[i];
    g.natoms = c->natoms[i];
    g.xyz = c->d_xyz.p + 3LL * c->atom_off[i];
    g.Z = c->d_Zd.p + c->atom_off[i];
    g.rad_r = x.rad_r.p;
    g.rad_w = x.rad_w.p;
    g.ang_u = x.ang_u.p;
    g.ang_w = x.ang_w.p;
    g.pts = nullptr;
    g.inv_sep = x.isep.p + x.isep_off[i];
    launch_xc_weight_grad(g, x.eg.p + x.pt_off[i], grad + 3LL * c->atom_off[i], st);
  }
  if (p2 >= 0) prof_end(c, p2, st);
  c->xc_launches[kXcGradWeight]++;
  HIPCHK(hipGetLastError());
}

void fock_build(bscf_ctx* c, double tau, int precision, bool masked, bool incremental = false) {
  ensure_work(c, tau, c->split_tol, precision == BSCF_MIXED);
  if (!c->fock_tuned[precision == BSCF_MIXED ? 1 : 0]) {
    // the autotuner times the cooperative forms too: lists with every item
    bool skipped = false;
    for (int q = 0; q < kNumQuartetClasses; ++q) skipped |= c->work[q].items_skipped;
    if (skipped) {
      c->items_all = true;
      build_work_host(c, tau, c->split_tol);
      build_work_device(c);
    }
    autotune_fock(c, precision == BSCF_MIXED ? 1 : 0);
  }
  const double t0 = now_ms();
  FockArgs a = fock_args(c, c->J.p, c->K.p, masked ? c->d_active.p : c->d_all_active.p);
  const BatchInfo bset = c->batch(masked);
  const bool det = c->det_now;
  const long long njk = (long long)c->max_ncd * (long long)c->kets.size();
  if (det) {
    if (c->Jfx.n < 2 * (size_t)c->mtot || c->Kfx.n < 2 * (size_t)c->mtot ||
        c->Jkfx.n < 2 * (size_t)std::max(njk, 1LL)) {
      c->Jfx.resize(2 * (size_t)c->mtot);
      c->Kfx.resize(2 * (size_t)c->mtot);
      c->Jkfx.resize(2 * (size_t)std::max(njk, 1LL));
      launch_fill_u64((long long)c->Jkfx.n, c->Jkfx.p, c->stream);
      incremental = false;   // fresh accumulators: this build starts from zero
      c->drop_fock_graphs();
    }
    a.Jfx = c->Jfx.p;
    a.Kfx = c->Kfx.p;
    a.Jkfx = c->Jkfx.p;
  }
  const int pcol = precision == BSCF_MIXED ? 1 : 0;
  auto alone = [&](int q) { return c->tune_ms[pcol][q][c->fock_variant[pcol][q]]; };
  // every launch of the J and K accumulation, in stream order (captured into
  // a graph or run directly)
  auto enqueue = [&]() {
  if (incremental) {
    launch_density_change(bset, c->max_n, c->P.p, c->Pprev.p, c->dP.p, c->d_dpmax.p, c->stream);
    // kept kets per row for the lane kernels, and the kept work of every
    // class counted on the device (the statistics read it later)
    // (one launch for all classes)
    const int pc = precision == BSCF_MIXED ? 1 : 0;
    const int ni = c->ninst;
    RowKeepClass rk[kNumQuartetClasses];
    int nrk = 0;
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      auto& W = c->work[q];
      if (!W.has_work) continue;
      RowKeepClass& r = rk[nrk++];
      r.cq = c->d_kept.p + (size_t)q * ni;
      r.cpq = c->d_kept.p + (size_t)(kNumQuartetClasses + q) * ni;
      r.block0 = 0;
      if (c->fock_variant[pc][q] == 1) {   // cooperative: counts over the item rows
        r.rows = W.d_rows.p;
        r.nrows = (int)W.rows.size();
        r.keep = nullptr;
        r.c32 = nullptr;
      } else {
        r.rows = W.ul.d_rows.p;
        r.nrows = (int)W.ul.rows.size();
        r.keep = W.ul.d_keep.p;
        r.c32 = lane_mode(c, precision, q) == 2
                    ? c->d_kept.p + (size_t)(2 * kNumQuartetClasses + q) * ni : nullptr;
      }
    }
    launch_row_keep(rk, nrk, c->d_kets.p, c->d_pairs.p, c->d_shells.p, c->d_Q.p, c->d_dpmax.p,
                    a.active, tau, ni, c->stream);
    a.P = c->dP.p;
    a.dpmax = c->d_dpmax.p;
    a.tau = tau;
    launch_shell_pmax(c->ninst, c->max_nshell, c->d_shell_off.p, c->d_nshell.p, c->d_pm_off.p,
                      c->d_shells.p, c->d_moff.p, c->d_nbf.p, c->dP.p, c->d_dpm.p, c->stream);
    a.dPm = c->d_dpm.p;
  } else if (det) {
    launch_fill_u64(2 * c->mtot, c->Jfx.p, c->stream);
    launch_fill_u64(2 * c->mtot, c->Kfx.p, c->stream);
  } else {
    launch_fill(c->J.p, c->mtot, 0.0, c->stream);
    launch_fill(c->K.p, c->mtot, 0.0, c->stream);
  }
  const KetPosArgs kp = ketpos_args(c);
  const QuartetClass* qc = quartet_classes();
  // class kernels run concurrently on the context stream and three auxiliary
  // streams, one per hardware queue (J and K are accumulated with atomics, so
  // their order does not matter): the longest first, each onto the stream with
  // the least time queued, so the first goes to the context stream, which
  // needs no cross-stream wait to start.  Kernels that need private scratch
  // stay on the context stream: the runtime reserves scratch per hardware
  // queue for full occupancy.
  constexpr int kRing = 4;
  const hipStream_t ring[kRing] = {c->stream, c->aux[0], c->aux[1], c->aux[2]};
  const int pbuild = c->profiling ? prof_begin(c, 0, 2, c->stream) : -1;
  launch_gather_pk(kp, c->max_ncd, a.P, c->d_Pk.p, c->stream);
  HIPCHK(hipEventRecord(c->ev_fork, c->stream));
  for (int k = 1; k < kRing; ++k) HIPCHK(hipStreamWaitEvent(ring[k], c->ev_fork, 0));
  // classes longest first (by the chosen kernel's time alone), each onto the
  // stream with the least time queued
  int order[kNumQuartetClasses];
  for (int q = 0; q < kNumQuartetClasses; ++q) order[q] = kNumQuartetClasses - 1 - q;
  std::stable_sort(order, order + kNumQuartetClasses,
                   [&](int x, int y) { return alone(x) > alone(y); });
  float load[kRing] = {};
  for (int q : order) {
    auto& W = c->work[q];
    if (!W.has_work) continue;
    // one launch: kernels with private scratch go to the context stream
    auto launch = [&](int pbytes, auto&& run) {
      int k = 0;
      if (pbytes == 0)
        for (int t = 1; t < kRing; ++t)
          if (load[t] < load[k]) k = t;
      load[k] += alone(q);
      const hipStream_t s = ring[k];
      const int pk = c->profiling ? prof_begin(c, q, 0, s) : -1;
      run(s);
      if (pk >= 0) prof_end(c, pk, s);
    };
    if (a.dPm) {   // this class's kept counts, lowered by what the kernels drop
      const size_t ni = (size_t)c->ninst;
      a.kept_q = c->d_kept.p + q * ni;
      a.kept_pq = c->d_kept.p + (kNumQuartetClasses + q) * ni;
      a.kept_32 = c->fock_variant[pcol][q] == 0 && lane_mode(c, precision, q) == 2
                      ? c->d_kept.p + (2 * kNumQuartetClasses + q) * ni : nullptr;
    }
    if (c->fock_variant[pcol][q] == 1) {
      set_class(a, W);
      launch(c->coop_bytes[q][0], [&](hipStream_t s) { qc[q].coop_fock(a, s); });
    } else {
      a.unit_threads = det ? 64 : c->unit_threads[pcol][q][c->fock_variant[pcol][q]];
      lane_launches(c, a, q, lane_mode(c, precision, q), [&](int k, auto&& run) {
        launch(c->private_bytes[q][k], run);
      });
    }
  }
  for (int k = 1; k < kRing; ++k) {   // ring[k] is aux[k - 1]
    HIPCHK(hipEventRecord(c->ev_join[k - 1], ring[k]));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join[k - 1], 0));
  }
  if (det) {
    launch_jk_finalize_fx(kp, c->max_ncd, c->Jkfx.p, c->Jfx.p, c->stream);
    launch_fx_to_double(c->mtot, c->Jfx.p, c->J.p, c->stream);
    launch_fx_to_double(c->mtot, c->Kfx.p, c->K.p, c->stream);
  } else {
    launch_jk_finalize(kp, c->max_ncd, c->d_Jk.p, c->J.p, c->stream);
  }
  if (pbuild >= 0) prof_end(c, pbuild, c->stream);
  };
  if (c->graph_fock && !c->profiling) {
    const auto key = std::make_tuple(pcol, masked ? 1 : 0, incremental ? 1 : 0, det ? 1 : 0, tau);
    auto g = c->fock_graphs.find(key);
    if (g == c->fock_graphs.end()) {
      HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipGraph_t graph = nullptr;
      try {
        enqueue();
      } catch (...) {
        (void)hipStreamEndCapture(c->stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      HIPCHK(hipStreamEndCapture(c->stream, &graph));
      c->graph_memset_nodes += memset_nodes(graph);
      hipGraphExec_t exec = nullptr;
      const hipError_t r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(r);
      g = c->fock_graphs.emplace(key, exec).first;
      c->fock_graph_captures++;
    }
    HIPCHK(hipGraphLaunch(g->second, c->stream));
    c->fock_graph_launches++;
  } else {
    enqueue();
  }
  HIPCHK(hipGetLastError());
  // work counts (an incremental build counts its kept work on the device)
  if (incremental) c->inc_builds++;
  for (int q = 0; q < kNumQuartetClasses; ++q) {
    auto& W = c->work[q];
    if (!W.has_work) continue;
    for (int i = 0; i < c->ninst; ++i)
      if (!masked || c->h_active[i]) W.screened_quart += W.inst_quart[i];
    if (!incremental)
      for (int i = 0; i < c->ninst; ++i)
        if (!masked || c->h_active[i]) {
          W.done_quart += W.inst_quart[i];
          W.done_primq += W.inst_primq[i];
          if (lane_mode(c, precision, q) == 2) W.done_quart32 += W.inst_quart32[i];
        }
    W.launches++;
  }
  if (c->prof_pending.size() > 8192) prof_collect(c);
  BatchInfo b = c->batch(masked);
  if (c->xc_now) {
    xc_build(c, c->P.p, masked);
    launch_fock_assemble(b, c->max_n, c->H.p, c->J.p, c->K.p, c->P.p, c->d_Enuc.p, c->F.p,
                         c->d_E.p, c->stream, kXcA0, c->xcs.V.p, c->xcs.exc.p);
  } else {
    launch_fock_assemble(b, c->max_n, c->H.p, c->J.p, c->K.p, c->P.p, c->d_Enuc.p, c->F.p,
                         c->d_E.p, c->stream);
  }
  launch_scale_copy(bset, c->max_n, c->P.p, c->Pprev.p, 1.0, 0, c->stream);   // next build's reference
  c->fock_builds++;
  c->t_fock_ms += now_ms() - t0;
}

void require_geom(bscf_ctx* c) {
  need(c->ninst > 0, BSCF_E_INVALID, "no instances set");
  need(c->have_geom, BSCF_E_INVALID, "no geometry set");
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* bscf_last_error(void) { return g_err.c_str(); }

bscf_status bscf_default_opts(bscf_scf_opts* o) {
  if (!o) return BSCF_E_INVALID;
  o->e_tol = 1e-8;
  o->comm_tol = 1e-6;
  o->schwarz_tol = 1e-12;
  o->fp32_split_tol = 1e-4;
  o->max_iter = 100;
  o->diis_size = 8;
  o->precision = BSCF_FP64;
  o->guess = BSCF_GUESS_CORE;
  o->deterministic = 0;
  o->density = BSCF_DENSITY_SP2;
  o->incremental = 1;
  o->graph = 1;
  return BSCF_OK;
}

bscf_status bscf_create(int hip_device, void* hip_stream, bscf_ctx** out) {
  return guard([&] {
    need(out != nullptr, BSCF_E_INVALID, "out is NULL");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    need(hip_device >= 0 && hip_device < ndev, BSCF_E_INVALID, "bad device index");
    std::unique_ptr<bscf_ctx> c(new bscf_ctx());
    c->device = hip_device;
    HIPCHK(hipSetDevice(hip_device));
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    for (int k = 0; k < bscf_ctx::kAux; ++k) {
      HIPCHK(hipStreamCreate(&c->aux[k]));
      HIPCHK(hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    {
      int lds = 0;
      HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device));
      c->max_lds_bytes = (size_t)lds;
    }
    {
      const QuartetClass* qc = quartet_classes();
      for (int q = 0; q < kNumQuartetClasses; ++q) {
        c->private_bytes[q][0] = qc[q].fock ? qc[q].fock_private_bytes(0) : 0;
        c->private_bytes[q][1] = qc[q].fock ? qc[q].fock_private_bytes(2) : 0;   // mixed form
        c->private_bytes[q][2] = qc[q].grad ? qc[q].grad_private_bytes() : 0;
        c->coop_bytes[q][0] = qc[q].coop_private_bytes(0);
        c->coop_bytes[q][1] = qc[q].coop_private_bytes(1);
        for (int k = 0; k < 3; ++k)
          need(c->private_bytes[q][k] >= 0, BSCF_E_DEVICE, "hipFuncGetAttributes failed");
        for (int k = 0; k < 2; ++k)
          need(c->coop_bytes[q][k] >= 0, BSCF_E_DEVICE, "hipFuncGetAttributes failed");
        c->fock_variant[0][q] = qc[q].fock && c->private_bytes[q][0] <= c->lane_scratch_max ? 0 : 1;
        c->fock_variant[1][q] = qc[q].fock && c->private_bytes[q][1] <= c->lane_scratch_max ? 0 : 1;
        c->grad_variant[q] = qc[q].grad && c->private_bytes[q][2] <= c->lane_scratch_max ? 0 : 1;
      }
    }
    mlp::init_noalloc_scratch(hip_device);
    BLASCHK(rocblas_create_handle(&c->blas));
    BLASCHK(rocblas_set_stream(c->blas, c->stream));
    std::vector<double> tab(kBoysRows * kBoysCols);
    boys_table_host(tab.data());
    std::vector<float> tab32(tab.begin(), tab.end());
    c->d_boys64.upload(tab, c->stream);
    c->d_boys32.upload(tab32, c->stream);
    sync(c.get());
    *out = c.release();
  });
}

bscf_status bscf_destroy(bscf_ctx* c) {
  if (!c) return BSCF_OK;
  if (c->work_job.valid()) {
    try {
      c->work_job.get();
    } catch (...) {
    }
  }
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (hipEvent_t e : c->prof_free) (void)hipEventDestroy(e);
  c->drop_graphs();
  if (c->blas) rocblas_destroy_handle(c->blas);
  for (int k = 0; k < bscf_ctx::kAux; ++k) {
    if (c->aux[k]) (void)hipStreamSynchronize(c->aux[k]);
    if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
    if (c->aux[k]) (void)hipStreamDestroy(c->aux[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  hipStream_t s = c->stream;
  bool own = c->own_stream;
  delete c;
  if (own) (void)hipStreamDestroy(s);
  return BSCF_OK;
}

bscf_status bscf_load_basis(bscf_ctx* c, const char* json) {
  return guard([&] {
    need(c && json, BSCF_E_INVALID, "NULL argument");
    join_work(c);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->drop_graphs();
    JParser p{json};
    JVal root = p.parse();
    const JVal* el = root.get("elements");
    need(el && el->kind == JVal::OBJ, BSCF_E_INVALID, "basis JSON: no 'elements' object");
    std::map<int, std::vector<BasisShell>> b;
    for (auto& kv : el->obj) {
      const JVal* z = kv.second.get("Z");
      const JVal* sh = kv.second.get("shells");
      need(z && sh && sh->kind == JVal::ARR, BSCF_E_INVALID, "basis JSON: element without Z/shells");
      std::vector<BasisShell> v;
      for (const JVal& s : sh->arr) {
        const JVal* l = s.get("l");
        const JVal* e = s.get("exponents");
        const JVal* d = s.get("coefficients");
        need(l && e && d && e->arr.size() == d->arr.size() && !e->arr.empty(), BSCF_E_INVALID,
             "basis JSON: malformed shell");
        const int ll = (int)l->num;
        need(ll >= 0 && ll <= kLmax, BSCF_E_UNSUPPORTED, "only s, p, d shells are supported");
        std::vector<double> ex, co;
        for (auto& x : e->arr) ex.push_back(x.num);
        for (auto& x : d->arr) co.push_back(x.num);
        for (double x : ex) need(x > 0.0, BSCF_E_INVALID, "non-positive exponent");
        v.push_back(normalise_shell(ll, ex, co));
      }
      b[(int)z->num] = v;
    }
    c->basis = b;
  });
}

bscf_status bscf_set_instances(bscf_ctx* c, int n_inst, const int* n_atoms, const int* Z,
                               const int* charge) {
  return guard([&] {
    need(c && n_inst > 0 && n_atoms && Z, BSCF_E_INVALID, "bad arguments");
    need(!c->basis.empty(), BSCF_E_INVALID, "load a basis first");
    // every argument is checked before the context changes, so a rejected
    // call leaves the previous instance set (and geometry) in place
    std::vector<int> ne_of(n_inst), nb_of(n_inst);
    int tot = 0;
    for (int i = 0; i < n_inst; ++i) {
      need(n_atoms[i] > 0, BSCF_E_INVALID, "instance without atoms");
      int ne = -(charge ? charge[i] : 0), nb = 0;
      for (int a = 0; a < n_atoms[i]; ++a) {
        const int z = Z[tot + a];
        auto it = c->basis.find(z);
        need(it != c->basis.end(), BSCF_E_UNSUPPORTED,
             "element Z=" + std::to_string(z) + " not in basis");
        ne += z;
        for (auto& s : it->second) nb += ncart(s.l);
      }
      need(ne > 0 && ne % 2 == 0, BSCF_E_UNSUPPORTED,
           "instance " + std::to_string(i) + ": closed-shell RHF needs an even electron count");
      need(ne / 2 <= nb, BSCF_E_UNSUPPORTED, "more occupied orbitals than basis functions");
      ne_of[i] = ne;
      nb_of[i] = nb;
      tot += n_atoms[i];
    }
    HIPCHK(hipSetDevice(c->device));
    join_work(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->drop_graphs();   // they hold addresses of buffers about to be resized
    // a device failure below leaves no instance set rather than host tables
    // that no longer match the device buffers
    struct Undo {
      bscf_ctx* c;
      bool done = false;
      ~Undo() {
        if (!done) {
          c->ninst = 0;
          c->have_geom = c->have_scf = c->have_C = false;
        }
      }
    } undo{c};
    c->have_geom = c->have_scf = c->have_C = false;
    c->ninst = n_inst;
    c->natoms.assign(n_atoms, n_atoms + n_inst);
    c->atom_off.assign(n_inst, 0);
    for (int i = 0, off = 0; i < n_inst; ++i) {
      c->atom_off[i] = off;
      off += n_atoms[i];
    }
    c->total_atoms = tot;
    c->Zs.assign(Z, Z + tot);
    c->charge.assign(n_inst, 0);
    if (charge) c->charge.assign(charge, charge + n_inst);
    c->nbf.assign(n_inst, 0);
    c->nocc.assign(n_inst, 0);
    c->moff.assign(n_inst, 0);
    c->mtot = 0;
    c->max_n = 0;
    c->max_atoms = 0;
    for (int i = 0; i < n_inst; ++i) {
      const int nb = nb_of[i];
      c->nbf[i] = nb;
      c->nocc[i] = ne_of[i] / 2;
      c->moff[i] = c->mtot;
      c->mtot += (long long)nb * nb;
      c->max_n = std::max(c->max_n, nb);
      c->max_atoms = std::max(c->max_atoms, n_atoms[i]);
    }
    c->groups.clear();
    for (int i = 0; i < n_inst; ++i) {
      if (!c->groups.empty() && c->groups.back().n == c->nbf[i] &&
          c->nocc[c->groups.back().first] == c->nocc[i])
        c->groups.back().count++;
      else
        c->groups.push_back(Group{i, 1, c->nbf[i]});
    }
    c->nprim_pairs = 0;
    build_shell_topology(c);
    const hipStream_t s = c->stream;
    c->d_nbf.upload(c->nbf, s);
    c->d_nocc.upload(c->nocc, s);
    c->d_moff.upload(c->moff, s);
    c->d_natoms.upload(c->natoms, s);
    c->d_atom_off.upload(c->atom_off, s);
    {
      std::vector<long long> po(c->ninst);
      long long t = 0;
      c->max_nshell = 0;
      for (int i = 0; i < c->ninst; ++i) {
        po[i] = t;
        t += (long long)c->nshell[i] * c->nshell[i];
        c->max_nshell = std::max(c->max_nshell, c->nshell[i]);
      }
      c->d_pm_off.upload(po, s);
      c->d_pmax.resize((size_t)std::max(t, 1LL));
      c->d_dpm.resize((size_t)std::max(t, 1LL));
      c->d_shell_off.upload(c->shell_off, s);
      c->d_nshell.upload(c->nshell, s);
    }
    std::vector<double> zd(c->Zs.begin(), c->Zs.end());
    c->d_Zd.upload(zd, s);
    c->d_sh_exp.upload(c->sh_exp, s);
    c->d_sh_coef.upload(c->sh_coef, s);
    c->d_pairs.upload(c->pairs, s);
    c->d_prim_owner.upload(c->prim_owner, s);
    c->d_prims.resize(c->nprim_pairs);
    c->d_Q.resize(c->pairs.size());
    c->d_pair_ids.clear();
    c->d_pair_ids.resize(kNumPairClasses);
    for (int pc = 0; pc < kNumPairClasses; ++pc) c->d_pair_ids[pc].upload(c->pairs_by_class[pc], s);
    // 1e task arrays: built per geometry (one_e_tasks)
    c->task_first.assign(kNumPairClasses, 0);
    c->task_count.assign(kNumPairClasses, 0);
    c->pair_rcut.clear();
    std::vector<int> ones(n_inst, 1), zeros(n_inst, 0);
    c->d_active.upload(ones, s);
    c->d_all_active.upload(ones, s);
    c->d_conv_iter.upload(zeros, s);
    c->d_status.upload(zeros, s);
    c->d_info.upload(zeros, s);
    const size_t mt = (size_t)c->mtot;
    for (DevBuf<double>* m : {&c->S, &c->T, &c->V, &c->H, &c->X, &c->F, &c->J, &c->K, &c->P,
                              &c->Pnew, &c->W, &c->tmp1, &c->tmp2, &c->err, &c->Fbar, &c->C,
                              &c->Cacc, &c->eig, &c->eigE, &c->Pprev, &c->dP, &c->Cprev,
                              &c->Cext, &c->Mpol})
      m->resize(mt);
    // a new batch has zero density until an SCF, a Fock build or
    // bscf_set_density gives it one (a user guess never starts from garbage)
    launch_fill(c->P.p, (long long)mt, 0.0, s);
    c->d_dpmax.resize((size_t)n_inst * (1 + (size_t)((c->max_n + 31) / 32) * ((c->max_n + 31) / 32)));
    c->d_kept.resize((size_t)3 * kNumQuartetClasses * n_inst);
    launch_fill(c->d_kept.p, (long long)c->d_kept.n, 0.0, s);
    c->Fhist.resize(mt * 8);
    c->Ehist.resize(mt * 8);
    c->diisB.resize((size_t)n_inst * 64);
    c->d_sp2.resize((size_t)(kSp2MaxSteps + 1) * 2 * n_inst * sp2_tiles(c->max_n));
    c->d_sp2b.resize((size_t)2 * n_inst * c->max_n);
    c->d_sp2c.resize((size_t)2 * n_inst);
    c->d_pin.resize((size_t)2 * n_inst);
    c->d_wmin.resize(n_inst);
    c->h_wmin.resize(n_inst);
    c->h_pin.resize((size_t)2 * n_inst);
    c->h_emax.resize(n_inst);
    c->d_omask.resize(n_inst);
    c->diisC.resize((size_t)n_inst * 8);
    c->diis_count.resize(n_inst);
    c->diis_head.resize(n_inst);
    c->d_Enuc.resize(n_inst);
    c->d_E.resize((size_t)n_inst * (1 + c->max_n));
    c->d_Eprev.resize(n_inst);
    c->d_emax.resize((size_t)n_inst * (1 + (size_t)((c->max_n + 31) / 32) * ((c->max_n + 31) / 32)));
    c->d_grad.resize((size_t)tot * 3);
    c->d_grad_tune.resize((size_t)tot * 3);
    c->d_xyz.resize((size_t)tot * 3);
    c->have_geom = false;
    c->have_scf = false;
    c->have_C = false;
    c->h_ccount.assign(n_inst, 0);
    c->d_cfirst.resize(n_inst);
    c->d_c2ok.resize(n_inst);
    c->work_tau = c->host_tau = -1.0;
    c->fock_tuned[0] = c->fock_tuned[1] = c->grad_tuned = false;
    c->items_all = false;
    c->guess.reset_batch(c->ninst);
    c->md.on = c->md.synced = c->md.have_force = false;
    c->str.on = c->str.synced = false;
    c->xcs.grid_ok = false;
    sync(c);
    undo.done = true;
  });
}

// The one-electron tasks of the current geometry: the shell pairs, grouped by
// pair class, whose centres lie within the pair's cutoff distance.  Past it
// every integral of the pair and its centre derivatives (S, T, V for every
// nucleus, their gradient) is below 1e-20: for R = |A - B| the bound
// sum_kl |c_k c_l| e^{-mu_kl R^2} (1 + R)^(la + lb + 2) (1 + 2 a_k)(1 + 2 b_l)
// max((pi/p)^1.5, 2 pi/p Z_max N_atoms) (mu = a b / p, p = a + b) covers the
// Gaussian products, the polynomial factors and the derivative factors; the
// cutoff is found once per pair by a 0.05-bohr scan of the bound's tail.
void one_e_tasks(bscf_ctx* c, hipStream_t s) {
  const size_t np = c->pairs.size();
  if (c->pair_rcut.size() != np) {
    c->pair_rcut.assign(np, 0.0);
    // shell types by their exact contents (l, exponents, coefficients)
    std::map<std::vector<double>, int> types;
    std::vector<int> type(c->shells.size());
    for (size_t k = 0; k < c->shells.size(); ++k) {
      const Shell& S = c->shells[k];
      std::vector<double> v{(double)S.l};
      for (int i = 0; i < S.nprim; ++i) {
        v.push_back(c->sh_exp[S.prim0 + i]);
        v.push_back(c->sh_coef[S.prim0 + i]);
      }
      type[k] = types.emplace(v, (int)types.size()).first->second;
    }
    std::vector<double> zn(c->ninst, 1.0);   // Z_max N_atoms per instance
    for (int i = 0; i < c->ninst; ++i) {
      double zmax = 1.0;
      for (int t = 0; t < c->natoms[i]; ++t) zmax = std::max(zmax, (double)c->Zs[c->atom_off[i] + t]);
      zn[i] = zmax * c->natoms[i];
    }
    std::map<std::array<double, 3>, double> cache;   // by (type a, type b, Z_max N_atoms)
    for (size_t k = 0; k < np; ++k) {
      const Shell& A = c->shells[c->pairs[k].a];
      const Shell& B = c->shells[c->pairs[k].b];
      const double zna = zn[A.inst];
      const std::array<double, 3> key = {(double)type[c->pairs[k].a], (double)type[c->pairs[k].b],
                                         zna};
      auto it = cache.find(key);
      if (it != cache.end()) {
        c->pair_rcut[k] = it->second;
        continue;
      }
      auto bound = [&](double R) {
        double b = 0.0;
        for (int i = 0; i < A.nprim; ++i)
          for (int j = 0; j < B.nprim; ++j) {
            const double al = c->sh_exp[A.prim0 + i], be = c->sh_exp[B.prim0 + j];
            const double p = al + be, mu = al * be / p;
            const double pre = std::max(std::pow(M_PI / p, 1.5), 2.0 * M_PI / p * zna);
            b += std::fabs(c->sh_coef[A.prim0 + i] * c->sh_coef[B.prim0 + j]) *
                 std::exp(-mu * R * R) * (1.0 + 2.0 * al) * (1.0 + 2.0 * be) * pre;
          }
        return b * std::pow(1.0 + R, A.l + B.l + 2);
      };
      double last = 0.0;
      for (double R = 0.0; R < 400.0; R += 0.05) {
        const double b = bound(R);
        if (b > 1e-20) last = R;
        else if (b < 1e-26) break;
      }
      c->pair_rcut[k] = last + 0.05;
      cache.emplace(key, last + 0.05);
    }
  }
  std::vector<int> ta, tb;
  ta.reserve(np);
  tb.reserve(np);
  for (int pc = 0; pc < kNumPairClasses; ++pc) {
    c->task_first[pc] = (int)ta.size();
    for (int pid : c->pairs_by_class[pc]) {
      const Shell& A = c->shells[c->pairs[pid].a];
      const Shell& B = c->shells[c->pairs[pid].b];
      const double dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
      const double rc = c->pair_rcut[pid];
      if (dx * dx + dy * dy + dz * dz > rc * rc) continue;
      ta.push_back(c->pairs[pid].a);
      tb.push_back(c->pairs[pid].b);
    }
    c->task_count[pc] = (int)ta.size() - c->task_first[pc];
  }
  c->d_task_a.upload(ta, s);
  c->d_task_b.upload(tb, s);
}

bscf_status bscf_set_geometries(bscf_ctx* c, const double* xyz) {
  return guard([&] {
    need(c && xyz, BSCF_E_INVALID, "NULL argument");
    need(c->ninst > 0, BSCF_E_INVALID, "set instances first");
    // checked first: a rejected geometry leaves the current one in place
    for (int k = 0; k < 3 * c->total_atoms; ++k)
      need(std::isfinite(xyz[k]), BSCF_E_INVALID, "non-finite coordinate");
    // from here on the context holds neither a geometry nor an SCF until the
    // call has finished: a device error part-way through cannot leave the
    // previous densities paired with the new coordinates
    c->have_geom = c->have_scf = false;
    c->md.synced = c->md.have_force = false;
    c->str.synced = false;
    c->xcs.grid_ok = false;
    HIPCHK(hipSetDevice(c->device));
    join_work(c);
    c->work_tau = c->host_tau = -1.0;
    const double t0 = now_ms();
    c->xyz.assign(xyz, xyz + 3 * c->total_atoms);
    for (Shell& s : c->shells) {
      s.x = xyz[3 * s.atom];
      s.y = xyz[3 * s.atom + 1];
      s.z = xyz[3 * s.atom + 2];
    }
    const hipStream_t st = c->stream;
    c->d_shells.upload(c->shells, st);
    c->d_xyz.upload(c->xyz, st);
    PrimPairSetupArgs pa{c->nprim_pairs, c->d_prim_owner.p, c->d_pairs.p, c->d_shells.p,
                         c->d_sh_exp.p, c->d_sh_coef.p, c->d_prims.p};
    launch_prim_pairs(pa, st);
    launch_nuclear(c->ninst, c->d_natoms.p, c->d_atom_off.p, c->d_xyz.p, c->d_Zd.p, c->d_Enuc.p,
                   nullptr, 0, st);
    // Schwarz bounds
    for (int pc = 0; pc < kNumPairClasses; ++pc) {
      if (c->pairs_by_class[pc].empty()) continue;
      SchwarzArgs sa{c->d_pair_ids[pc].p, (int)c->pairs_by_class[pc].size(), c->d_pairs.p,
                     c->d_prims.p, c->d_shells.p, c->d_boys64.p, c->d_Q.p};
      const int la = pc == 0 ? 0 : (pc < 3 ? 1 : 2);
      const int lb = pc - la * (la + 1) / 2;
      schwarz_launcher(la, lb)(sa, st);
    }
    // one-electron matrices over the pairs that are not negligible at this
    // geometry (the others stay zero)
    one_e_tasks(c, st);
    launch_fill(c->S.p, c->mtot, 0.0, st);
    launch_fill(c->T.p, c->mtot, 0.0, st);
    launch_fill(c->V.p, c->mtot, 0.0, st);
    for (int pc = 0; pc < kNumPairClasses; ++pc) {
      if (c->task_count[pc] == 0) continue;
      const int la = pc == 0 ? 0 : (pc < 3 ? 1 : 2);
      const int lb = pc - la * (la + 1) / 2;
      OneEArgs oa;
      oa.ntasks = c->task_count[pc];
      oa.task_a = c->d_task_a.p + c->task_first[pc];
      oa.task_b = c->d_task_b.p + c->task_first[pc];
      oa.shells = c->d_shells.p;
      oa.sh_exp = c->d_sh_exp.p;
      oa.sh_coef = c->d_sh_coef.p;
      oa.natoms = c->d_natoms.p;
      oa.atom_off = c->d_atom_off.p;
      oa.atom_xyz = c->d_xyz.p;
      oa.atom_Z = c->d_Zd.p;
      oa.nbf = c->d_nbf.p;
      oa.moff = c->d_moff.p;
      oa.boys64 = c->d_boys64.p;
      oa.S = c->S.p;
      oa.T = c->T.p;
      oa.V = c->V.p;
      launch_onee(la, lb, oa, st);
    }
    HIPCHK(hipGetLastError());
    // H = T + V
    BatchInfo ball = c->batch(false);
    launch_scale_copy(ball, c->max_n, c->T.p, c->H.p, 1.0, 0, st);
    {
      const double one = 1.0;
      BLASCHK(rocblas_daxpy(c->blas, (int)c->mtot, &one, c->V.p, 1, c->H.p, 1));
    }
    // Schwarz bounds to the host; the screened work lists are then built on a
    // worker thread while the stream computes the orthogonaliser (and the
    // caller's SCF its guess); the first Fock build joins it
    c->Q.resize(c->pairs.size());
    HIPCHK(hipMemcpyAsync(c->Q.data(), c->d_Q.p, c->pairs.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    sync(c);
    const double split = c->split_tol;
    c->work_job = std::async(std::launch::async, [c, split] { build_work_host(c, 1e-12, split); });
    build_orthogonaliser(c);
    c->have_geom = true;
    c->have_scf = false;
    c->t_setup_ms += now_ms() - t0;
  });
}

bscf_status bscf_build_jk(bscf_ctx* c, const double* P, double* J, double* K, double tau,
                          int precision, int device_ptrs) {
  return guard([&] {
    need(c && P && J && K, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    const auto kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    c->have_scf = false;   // the SCF density is replaced: forces need a new SCF
    HIPCHK(hipMemcpyAsync(c->P.p, P, c->mtot * sizeof(double), kind, c->stream));
    c->det_now = c->det;
    c->xc_now = 0;
    fock_build(c, tau, precision, false);
    // symmetrised J, K
    BatchInfo b = c->batch(false);
    launch_scale_copy(b, c->max_n, c->J.p, c->tmp1.p, 0.5, 1, c->stream);
    launch_scale_copy(b, c->max_n, c->K.p, c->tmp2.p, 0.5, 1, c->stream);
    const double half = 0.5;
    BLASCHK(rocblas_daxpy(c->blas, (int)c->mtot, &half, c->J.p, 1, c->tmp1.p, 1));
    BLASCHK(rocblas_daxpy(c->blas, (int)c->mtot, &half, c->K.p, 1, c->tmp2.p, 1));
    const auto back = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(J, c->tmp1.p, c->mtot * sizeof(double), back, c->stream));
    HIPCHK(hipMemcpyAsync(K, c->tmp2.p, c->mtot * sizeof(double), back, c->stream));
    sync(c);
  });
}

bscf_status bscf_build_fock(bscf_ctx* c, const double* P, double* F, double* E, double tau,
                            int precision, int device_ptrs) {
  return guard([&] {
    need(c && P && F, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    const auto kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    c->have_scf = false;   // the SCF density is replaced: forces need a new SCF
    HIPCHK(hipMemcpyAsync(c->P.p, P, c->mtot * sizeof(double), kind, c->stream));
    c->det_now = c->det;
    c->xc_now = c->xc;
    fock_build(c, tau, precision, false);
    const auto back = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(F, c->F.p, c->mtot * sizeof(double), back, c->stream));
    if (E) HIPCHK(hipMemcpyAsync(E, c->d_E.p, c->ninst * sizeof(double), device_ptrs ? back : hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

bscf_status bscf_set_density(bscf_ctx* c, const double* P, int device_ptrs) {
  return guard([&] {
    need(c && P, BSCF_E_INVALID, "NULL argument");
    need(c->ninst > 0, BSCF_E_INVALID, "set instances first");
    c->have_scf = false;   // the SCF density is replaced: forces need a new SCF
    HIPCHK(hipMemcpyAsync(c->P.p, P, c->mtot * sizeof(double),
                          device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    sync(c);
  });
}

namespace {
// out[o + j*no + i] = U[o + j*no + i] * w[o + j]^{-1/2}, no x no column-major blocks
__global__ void scale_cols_occ_kernel(int ninst, const long long* moff, const int* nocc,
                                      const double* U, const double* w, double* out) {
  const int inst = blockIdx.y;
  if (inst >= ninst) return;
  const int no = nocc[inst];
  const long long o = moff[inst], nn = (long long)no * no;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x)
    out[o + k] = U[o + k] / sqrt(w[o + k / no]);
}

// previous-step guess: C_occ' = C_occ (C_occ^T S C_occ)^{-1/2}, P = 2 C' C'^T,
// with C_occ the first nocc columns of Csrc (default: the last SCF's orbitals)
void previous_guess(bscf_ctx* c, const double* Csrc = nullptr) {
  if (!Csrc) Csrc = c->Cacc.p;
  const double one = 1.0, zero = 0.0, two = 2.0;
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int n = g.n, no = c->nocc[g.first];
    // tmp1 = S C_occ (n x no)
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none,
                                          n, no, n, &one, c->S.p + o, n, st, Csrc + o, n, st,
                                          &zero, c->tmp1.p + o, n, st, g.count));
    // eig = C_occ^T S C_occ (no x no, leading dim no)
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose,
                                          rocblas_operation_none, no, no, n, &one, Csrc + o,
                                          n, st, c->tmp1.p + o, n, st, &zero, c->eig.p + o, no, st,
                                          g.count));
    BLASCHK(rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper,
                                             no, c->eig.p + o, no, st, c->tmp2.p + o, st,
                                             c->eigE.p + o, st, c->d_info.p + g.first, g.count));
  }
  const long long nn = (long long)c->max_n * c->max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(scale_cols_occ_kernel, dim3(gx, c->ninst), dim3(256), 0, c->stream, c->ninst,
                     c->d_moff.p, c->d_nocc.p, c->eig.p, c->tmp2.p, c->err.p);
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int n = g.n, no = c->nocc[g.first];
    // Minv = (U w^-1/2) U^T -> Fbar (no x no)
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                          rocblas_operation_transpose, no, no, no, &one,
                                          c->err.p + o, no, st, c->eig.p + o, no, st, &zero,
                                          c->Fbar.p + o, no, st, g.count));
    // C' = C_occ Minv (n x no) -> tmp1
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none,
                                          n, no, no, &one, Csrc + o, n, st, c->Fbar.p + o, no,
                                          st, &zero, c->tmp1.p + o, n, st, g.count));
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                          rocblas_operation_transpose, n, n, no, &two,
                                          c->tmp1.p + o, n, st, c->tmp1.p + o, n, st, &zero,
                                          c->P.p + o, n, st, g.count));
  }
}

// C2 U - 2 C1 -> -(C_ext) for the instances with two stored SCFs (c2ok), C1
// otherwise: out = c2ok ? 2 C1 - C2U : C1 over the first nocc columns
__global__ void extrap_kernel(int ninst, const long long* moff, const int* nbf, const int* nocc,
                              const int* c2ok, const double* C1, const double* C2U, double* out) {
  const int inst = blockIdx.y;
  if (inst >= ninst) return;
  const long long o = moff[inst], m = (long long)nbf[inst] * nocc[inst];
  const bool ex = c2ok[inst] != 0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < m;
       k += (long long)gridDim.x * blockDim.x)
    out[o + k] = ex ? 2.0 * C1[o + k] - C2U[o + k] : C1[o + k];
}

// Second-order orbital extrapolation (BSCF_GUESS_EXTRAPOLATED): align the
// orbitals before the last (C2) to the last (C1) by the orthogonal Procrustes
// rotation U = M (M^T M)^{-1/2}, M = C2^T S C1 (occupied columns, current S),
// take C = 2 C1 - C2 U and re-orthonormalise it as the previous-step guess.
void extrapolated_guess(bscf_ctx* c) {
  const double one = 1.0, zero = 0.0;
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int n = g.n, no = c->nocc[g.first];
    // tmp1 = S C1 (n x no); Mpol = C2^T tmp1 (no x no); eig = Mpol^T Mpol
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none,
                                          n, no, n, &one, c->S.p + o, n, st, c->Cacc.p + o, n, st,
                                          &zero, c->tmp1.p + o, n, st, g.count));
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose,
                                          rocblas_operation_none, no, no, n, &one, c->Cprev.p + o,
                                          n, st, c->tmp1.p + o, n, st, &zero, c->Mpol.p + o, no, st,
                                          g.count));
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose,
                                          rocblas_operation_none, no, no, no, &one, c->Mpol.p + o,
                                          no, st, c->Mpol.p + o, no, st, &zero, c->eig.p + o, no, st,
                                          g.count));
    BLASCHK(rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper,
                                             no, c->eig.p + o, no, st, c->tmp2.p + o, st,
                                             c->eigE.p + o, st, c->d_info.p + g.first, g.count));
  }
  const long long nn = (long long)c->max_n * c->max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(scale_cols_occ_kernel, dim3(gx, c->ninst), dim3(256), 0, c->stream, c->ninst,
                     c->d_moff.p, c->d_nocc.p, c->eig.p, c->tmp2.p, c->err.p);
  for (const Group& g : c->groups) {
    const long long o = c->moff[g.first];
    const long long st = (long long)g.n * g.n;
    const int n = g.n, no = c->nocc[g.first];
    // (M^T M)^{-1/2} = (V w^-1/2) V^T -> Fbar; U = Mpol Fbar -> tmp2; C2 U -> Cext
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                          rocblas_operation_transpose, no, no, no, &one,
                                          c->err.p + o, no, st, c->eig.p + o, no, st, &zero,
                                          c->Fbar.p + o, no, st, g.count));
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none,
                                          no, no, no, &one, c->Mpol.p + o, no, st, c->Fbar.p + o,
                                          no, st, &zero, c->tmp2.p + o, no, st, g.count));
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none,
                                          n, no, no, &one, c->Cprev.p + o, n, st, c->tmp2.p + o,
                                          no, st, &zero, c->Cext.p + o, n, st, g.count));
  }
  hipLaunchKernelGGL(extrap_kernel, dim3(gx, c->ninst), dim3(256), 0, c->stream, c->ninst,
                     c->d_moff.p, c->d_nbf.p, c->d_nocc.p, c->d_c2ok.p, c->Cacc.p, c->Cext.p,
                     c->Cext.p);
  HIPCHK(hipGetLastError());
  previous_guess(c, c->Cext.p);
}

mlp::Batch guess_batch(bscf_ctx* c) {
  mlp::Batch b;
  b.ninst = c->ninst;
  b.moff = c->moff.data();
  b.nbf = c->nbf.data();
  b.natoms = c->natoms.data();
  b.atom_off = c->atom_off.data();
  b.Z = c->Zs.data();
  b.xyz = c->xyz.data();
  b.atom_bf0 = c->atom_bf0.data();
  b.atom_nbf = c->atom_nbf.data();
  b.total_atoms = c->total_atoms;
  b.mtot = (size_t)c->mtot;
  b.P = c->P.p;
  b.stream = c->stream;
  return b;
}

// dst <- src for the active instances; the orbitals dst held move to prev
// (or, for an instance without stored orbitals (first), src itself)
__global__ void commit_C_kernel(BatchInfo b, const int* first, const double* src, double* dst,
                                double* prev) {
  const int inst = blockIdx.y;
  if (!b.active[inst]) return;
  const int n = b.nbf[inst];
  const long long o = b.moff[inst], nn = (long long)n * n;
  const bool f = first[inst] != 0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    const double old = dst[o + k];
    prev[o + k] = f ? src[o + k] : old;
    dst[o + k] = src[o + k];
  }
}
}  // namespace

bscf_status bscf_run_scf(bscf_ctx* c, const bscf_scf_opts* opts, double* E, int* n_iter,
                         int* status) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    bscf_scf_opts o;
    bscf_default_opts(&o);
    if (opts) o = *opts;
    need(o.max_iter > 0 && o.diis_size >= 1 && o.diis_size <= 8, BSCF_E_INVALID, "bad options");
    need(o.guess >= BSCF_GUESS_CORE && o.guess <= BSCF_GUESS_EXTRAPOLATED, BSCF_E_INVALID,
         "guess must be a bscf_guess");
    need(o.fp32_split_tol > 0.0, BSCF_E_INVALID, "fp32_split_tol must be positive");
    need(o.density == BSCF_DENSITY_SP2 || o.density == BSCF_DENSITY_EIG, BSCF_E_INVALID,
         "density must be BSCF_DENSITY_SP2 or BSCF_DENSITY_EIG");
    need(o.deterministic == 0 || o.deterministic == 1, BSCF_E_INVALID, "deterministic must be 0 or 1");
    need(o.graph >= 0 && o.graph <= 2, BSCF_E_INVALID, "graph must be 0, 1 or 2");
    // graph 2: this call's Fock builds replay captured J and K launches
    struct FockGraphs {
      bscf_ctx* c;
      ~FockGraphs() { c->graph_fock = 0; }
    } fg{c};
    c->graph_fock = o.graph == 2 ? 1 : 0;
    c->det_now = o.deterministic == 1 || c->det;
    c->xc_now = c->xc;
    c->scf_xc = c->xc != 0;
    c->split_tol = o.fp32_split_tol;
    c->have_scf = false;   // set again once every instance has its density
    const double t0 = now_ms();
    const hipStream_t st = c->stream;
    const int ni = c->ninst;
    std::vector<int> flags(ni, 1), stat(ni, 1), iters(ni, 0), updates(ni, 0);
    c->h_active.assign(ni, 1);
    // guess
    int guess = o.guess;
    std::vector<int> fallback(ni, 0);
    const mlp::Batch gb = guess_batch(c);
    // the learned guess corrects the previous-step guess; without previous
    // orbitals both fall back to the core guess
    if ((guess == BSCF_GUESS_PREVIOUS || guess == BSCF_GUESS_LEARNED ||
         guess == BSCF_GUESS_EXTRAPOLATED) && !c->have_C) {
      if (guess == BSCF_GUESS_LEARNED) std::fill(fallback.begin(), fallback.end(), BSCF_FALLBACK_USED);
      guess = BSCF_GUESS_CORE;
    }
    if (guess == BSCF_GUESS_CORE) {
      c->d_active.upload(flags, st);
      density_from_fock(c, c->H.p, c->batch(true), flags, o.density, c->P.p);
      c->guess.begin_step(gb, false);
    } else if (guess == BSCF_GUESS_EXTRAPOLATED) {
      // the extrapolated orbitals where two SCFs are stored (the previous
      // step's elsewhere)
      std::vector<int> ok(ni);
      for (int i = 0; i < ni; ++i) ok[i] = c->h_ccount[i] >= 2 ? 1 : 0;
      c->d_c2ok.upload(ok, st);
      extrapolated_guess(c);
      c->guess.begin_step(gb, true);
    } else if (guess == BSCF_GUESS_PREVIOUS || guess == BSCF_GUESS_LEARNED) {
      // the learned guess corrects the previous-step density (its network
      // carries last step's residual forward, which that base keeps coherent)
      previous_guess(c);
      c->guess.begin_step(gb, true);
      if (guess == BSCF_GUESS_LEARNED && !c->guess.predict(gb))
        std::fill(fallback.begin(), fallback.end(), BSCF_FALLBACK_USED);
    } else {
      c->guess.begin_step(gb, false);   // BSCF_GUESS_USER: P already set
    }
    c->d_active.upload(flags, st);
    c->d_status.upload(stat, st);
    std::vector<int> zeros(ni, 0);
    c->diis_count.upload(zeros, st);
    c->diis_head.upload(zeros, st);
    c->d_conv_iter.upload(zeros, st);
    launch_fill(c->diisB.p, (long long)ni * 64, 0.0, st);
    DiisArgs d;
    d.ninst = ni;
    d.max_vec = o.diis_size;
    d.nbf = c->d_nbf.p;
    d.moff = c->d_moff.p;
    d.active = c->d_active.p;
    d.stride = c->mtot;
    d.Fhist = c->Fhist.p;
    d.Ehist = c->Ehist.p;
    d.B = c->diisB.p;
    d.count = c->diis_count.p;
    d.head = c->diis_head.p;
    d.coef = c->diisC.p;
    BatchInfo bm = c->batch(true);
    int it = 0;
    int since_full = 0;          // incremental builds since the last full one
    bool stalled = false;        // full builds from here on
    std::vector<double> err_hist[3];
    for (auto& h : err_hist) h.assign(ni, 0.0);
    for (; it < o.max_iter; ++it) {
      const bool full = it == 0 || since_full + 1 >= kFullEvery || stalled;
      fock_build(c, o.schwarz_tol, o.precision, true, o.incremental && !full);
      since_full = full ? 0 : since_full + 1;
      // the rest of the iteration goes out before the host knows which
      // replicas this iteration finishes (density_half); one synchronisation
      // per iteration then reads the active flags and whether every SP2
      // projection finished
      const int k = o.density == BSCF_DENSITY_SP2 ? sp2_target(c, sp2_slot(it)) : -1;
      if (k >= 0 && o.graph) density_half_graph(c, o, d, bm, k);
      else density_half(c, o, d, bm, k);
      HIPCHK(hipMemcpyAsync(c->h_pin.p, c->d_pin.p, (k >= 0 ? 2 : 1) * ni * sizeof(int),
                            hipMemcpyDeviceToHost, st));
      if (o.incremental)
        HIPCHK(hipMemcpyAsync(c->h_emax.p, c->d_emax.p, ni * sizeof(double),
                              hipMemcpyDeviceToHost, st));
      sync(c);
      if (o.incremental) {
        std::swap(err_hist[0], err_hist[1]);
        std::swap(err_hist[1], err_hist[2]);
        for (int i = 0; i < ni && !stalled; ++i) {
          // instances active in this iteration and not finished by it (the
          // others' errors are stale or no longer matter)
          if (!(flags[i] && c->h_pin.p[i])) {
            err_hist[2][i] = 0.0;
            continue;
          }
          const double e = c->h_emax.p[i];
          err_hist[2][i] = e;
          if (it >= 2 && since_full >= 2 && e < kStallNear * o.comm_tol &&
              e >= kStallRatio * err_hist[0][i] && err_hist[0][i] > 0.0)
            stalled = true;
        }
      }
      std::copy(c->h_pin.p, c->h_pin.p + ni, flags.begin());
      c->scf_iters++;
      c->h_active = flags;
      bool any = false;
      for (int i = 0; i < ni; ++i) any |= flags[i] != 0;
      if (!any) break;
      if (k >= 0) {
        // a projection still short of its need is finished here, or falls
        // back to the eigenvector route when it has no gap
        int ks = k;
        if (!sp2_finished(c, flags, ks, sp2_slot(it))) {
          if (!sp2_extend(c, bm, flags, sp2_slot(it), ks, c->Pnew.p)) {
            c->sp2_fallbacks++;
            orbitals_from_fock(c, c->Fbar.p);
            density_from_orbitals(c, c->Pnew.p);
          }
          launch_commit(bm, c->max_n, c->Pnew.p, c->P.p, st);
        }
        c->sp2_calls++;
        c->sp2_steps += ks;
      }
      for (int i = 0; i < ni; ++i) updates[i] += flags[i] != 0;
    }
    // orbitals for the next call's previous-step guess, once per call: those
    // of the Fock matrix each replica's final density came from (DIIS leaves a
    // finished replica's Fbar alone); a replica without a density update here
    // keeps its stored orbitals
    {
      std::vector<int> mask(ni);
      bool anyu = false;
      for (int i = 0; i < ni; ++i) anyu |= (mask[i] = updates[i] > 0) != 0;
      if (anyu) {
        c->d_omask.upload(mask, st);
        orbitals_from_fock(c, c->Fbar.p);
        BatchInfo bo = c->batch(false);
        bo.active = c->d_omask.p;
        std::vector<int> first(ni);
        for (int i = 0; i < ni; ++i) first[i] = c->h_ccount[i] == 0 ? 1 : 0;
        c->d_cfirst.upload(first, st);
        commit_C_kernel<<<dim3(1024, ni), 256, 0, st>>>(bo, c->d_cfirst.p, c->C.p, c->Cacc.p,
                                                         c->Cprev.p);
        for (int i = 0; i < ni; ++i)
          if (mask[i]) c->h_ccount[i] = std::min(2, c->h_ccount[i] + 1);
      }
    }
    std::vector<double> e(ni);
    HIPCHK(hipMemcpyAsync(e.data(), c->d_E.p, ni * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(stat.data(), c->d_status.p, ni * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(iters.data(), c->d_conv_iter.p, ni * sizeof(int), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int i = 0; i < ni; ++i) {
      if (iters[i] == 0) iters[i] = it < o.max_iter ? it + 1 : o.max_iter;
      stat[i] |= fallback[i];
    }
    if (E) std::copy(e.begin(), e.end(), E);
    if (n_iter) std::copy(iters.begin(), iters.end(), n_iter);
    if (status) std::copy(stat.begin(), stat.end(), status);
    c->last_iters = iters;
    c->have_C = true;
    c->have_scf = true;
    c->guess.record(guess_batch(c));
    c->t_scf_ms += now_ms() - t0;
  });
}

namespace {
// -dE/dR of every instance at the densities c->P and Fock matrices c->F
// (W = P F P / 2) into Fout [total_atoms][3] (host)
// with_xc: B3LYP forces (exact exchange scaled by the hybrid's share, plus
// the exchange-correlation term); W comes from the Kohn-Sham F then
void forces_impl(bscf_ctx* c, double* Fout, bool with_xc = false) {
    const double t0 = now_ms();
    const hipStream_t st = c->stream;
    // W = P F P / 2
    gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 1.0, c->P.p, c->F.p, 0.0,
         c->tmp1.p);
    gemm(c, rocblas_operation_none, rocblas_operation_none, -1, -1, -1, 0.5, c->tmp1.p, c->P.p, 0.0,
         c->W.p);
    launch_fill(c->d_grad.p, 3LL * c->total_atoms, 0.0, st);
    launch_nuclear(c->ninst, c->d_natoms.p, c->d_atom_off.p, c->d_xyz.p, c->d_Zd.p, c->d_Enuc.p,
                   c->d_grad.p, 1, st);
    // one-electron gradient arguments per pair class (launched below with the
    // two-electron classes)
    Grad1EArgs g1[kNumPairClasses];
    for (int pc = 0; pc < kNumPairClasses; ++pc) {
      Grad1EArgs& g = g1[pc];
      g.ntasks = c->task_count[pc];
      g.task_a = c->d_task_a.p + c->task_first[pc];
      g.task_b = c->d_task_b.p + c->task_first[pc];
      g.shells = c->d_shells.p;
      g.sh_exp = c->d_sh_exp.p;
      g.sh_coef = c->d_sh_coef.p;
      g.natoms = c->d_natoms.p;
      g.atom_off = c->d_atom_off.p;
      g.atom_xyz = c->d_xyz.p;
      g.atom_Z = c->d_Zd.p;
      g.nbf = c->d_nbf.p;
      g.moff = c->d_moff.p;
      g.boys64 = c->d_boys64.p;
      g.P = c->P.p;
      g.W = c->W.p;
      g.active = c->d_all_active.p;
      g.grad = c->d_grad.p;
    }
    auto pc_l = [](int pc, int& la, int& lb) {
      la = pc == 0 ? 0 : (pc < 3 ? 1 : 2);
      lb = pc - la * (la + 1) / 2;
    };
    // two-electron part over the same screened work lists
    GradArgs ga;
    ga.items = nullptr;
    ga.nitems = 0;
    ga.rows = nullptr;
    ga.units = nullptr;
    ga.nunits = 0;
    ga.urows = nullptr;
    ga.pairs = c->d_pairs.p;
    ga.prims = c->d_prims.p;
    ga.shells = c->d_shells.p;
    ga.kets = c->d_kets.p;
    ga.kprims = c->d_kprims.p;
    ga.kpos = c->d_kpos.p;
    ga.max_prims = c->max_prims;
    ga.moff = c->d_moff.p;
    ga.nbf = c->d_nbf.p;
    ga.atom_off = c->d_atom_off.p;
    ga.nmax = c->max_n;
    ga.max_atoms = c->max_atoms;
    ga.nk_total = (int)c->kets.size();
    ga.P = c->P.p;
    ga.Pk = c->d_Pk.p;
    ga.grad = c->d_grad.p;
    ga.boys64 = c->d_boys64.p;
    ga.unit_threads = 64;
    // density-weighted screening at the lists' Schwarz cutoff
    ga.Q = c->d_Q.p;
    ga.Pm = c->d_pmax.p;
    ga.pm_off = c->d_pm_off.p;
    ga.shell_off = c->d_shell_off.p;
    ga.nsh = c->d_nshell.p;
    ga.tau = c->work_tau;
    ga.kx = with_xc ? kXcA0 : 1.0;
    c->d_gstat.resize((size_t)2 * kNumQuartetClasses);
    launch_fill(c->d_gstat.p, 2LL * kNumQuartetClasses, 0.0, st);
    ga.gstat = nullptr;
    launch_shell_pmax(c->ninst, c->max_nshell, c->d_shell_off.p, c->d_nshell.p, c->d_pm_off.p,
                      c->d_shells.p, c->d_moff.p, c->d_nbf.p, c->P.p, c->d_pmax.p, st);
    launch_gather_pk(ketpos_args(c), c->max_ncd, c->P.p, c->d_Pk.p, st);
    auto set_gclass = [](GradArgs& g, const bscf_ctx::ClassWork& W) {
      g.items = W.d_items.p;
      g.nitems = (int)W.items.size();
      g.rows = W.d_rows.p;
      g.units = W.ul.d_units.p;
      g.nunits = (int)W.ul.units.size();
      g.urows = W.ul.d_rows.p;
      g.max_prims = W.max_prims;
    };
    const QuartetClass* qc = quartet_classes();
    if (!c->grad_tuned) {
      // time both gradient variants where both exist, and every kernel that
      // the gradient launches alone (into a throwaway buffer): the choice
      // of variant and the stream schedule below use these times
      const char* env = getenv("BSCF_VARIANT");
      const char* env_u = getenv("BSCF_UNIT_THREADS");
      const int env_nt = env_u ? atoi(env_u) : 0;
      need(env_nt == 0 || env_nt == 64 || env_nt == 128 || env_nt == 256, BSCF_E_INVALID,
           "BSCF_UNIT_THREADS must be 64, 128 or 256");
      // the kernels add into grad[3 * atom + d] of every atom of the batch
      need(c->d_grad_tune.n >= (size_t)3 * c->total_atoms, BSCF_E_STATE,
           "gradient timing buffer smaller than the batch");
      GradArgs gt = ga;
      gt.grad = c->d_grad_tune.p;
      gt.gstat = nullptr;
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      auto time_alone = [&](auto&& run) {
        HIPCHK(hipEventRecord(e0, st));
        run();
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        return ms;
      };
      for (int q = 0; q < kNumQuartetClasses; ++q) {
        auto& W = c->work[q];
        c->tune_grad_ms[q][0] = c->tune_grad_ms[q][1] = 0.0f;
        if (!W.has_work) continue;
        set_gclass(gt, W);
        const bool lds_ok = sizeof(double) * (size_t)grad_unit_lds_doubles(
                                qc[q].la, qc[q].lb, c->max_n, c->max_atoms, W.max_prims) <=
                            c->max_lds_bytes;
        const bool lane_ok = qc[q].grad && lds_ok && c->private_bytes[q][2] <= c->lane_scratch_max;
        c->grad_unit_threads[q] = 64;
        if (lane_ok && !(env && !strcmp(env, "coop"))) {
          // units of one, two and four wavefronts, the fastest kept
          float best = -1.0f;
          for (int nt : {64, 128, 256}) {
            if (env_nt > 0 && nt != env_nt) continue;
            gt.unit_threads = nt;
            const float ms = time_alone([&] { qc[q].grad(gt, st); });
            if (best < 0.0f || ms < best) {
              best = ms;
              c->grad_unit_threads[q] = nt;
            }
          }
          gt.unit_threads = 64;
          c->tune_grad_ms[q][0] = best;
        }
        if (!lane_ok || !(env && !strcmp(env, "lane")))
          c->tune_grad_ms[q][1] = time_alone([&] { qc[q].coop_grad(gt, st); });
        if (!lane_ok) c->grad_variant[q] = 1;
        else if (env && !strcmp(env, "lane")) c->grad_variant[q] = 0;
        else if (env && !strcmp(env, "coop")) c->grad_variant[q] = 1;
        else c->grad_variant[q] = c->tune_grad_ms[q][1] < c->tune_grad_ms[q][0] ? 1 : 0;
      }
      for (int pc = 0; pc < kNumPairClasses; ++pc) {
        c->tune_grad1e_ms[pc] = 0.0f;
        if (g1[pc].ntasks == 0) continue;
        Grad1EArgs g = g1[pc];
        g.grad = c->d_grad_tune.p;
        int la, lb;
        pc_l(pc, la, lb);
        c->tune_grad1e_ms[pc] = time_alone([&] { launch_grad1e(la, lb, g, st); });
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      c->grad_tuned = true;
    }
    // Every class kernel and one-electron kernel is independent (the force
    // accumulates with atomics): longest first, each onto the stream with the
    // least time queued so far (the context stream and the auxiliary ones),
    // from the times alone above.  Kernels with private scratch stay on the
    // context stream: the runtime reserves scratch per hardware queue.
    struct Job {
      float ms;
      int q;    // quartet class, or -1 - pair class for a one-electron kernel
      int pbytes;
    };
    std::vector<Job> jobs;
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      if (!c->work[q].has_work) continue;
      const int var = c->grad_variant[q];
      jobs.push_back({c->tune_grad_ms[q][var], q,
                      var ? c->coop_bytes[q][1] : c->private_bytes[q][2]});
    }
    for (int pc = 0; pc < kNumPairClasses; ++pc)
      if (g1[pc].ntasks > 0) jobs.push_back({c->tune_grad1e_ms[pc], -1 - pc, 0});
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& x, const Job& y) { return x.ms > y.ms; });
    constexpr int kNs = 4;   // one stream per hardware queue (five measured slower)
    const hipStream_t ring[kNs] = {st, c->aux[0], c->aux[1], c->aux[2]};
    float load[kNs] = {};
    bool used[kNs] = {true};
    HIPCHK(hipEventRecord(c->ev_fork, st));
    for (const Job& j : jobs) {
      int k = 0;
      if (j.pbytes == 0)
        for (int t = 1; t < kNs; ++t)
          if (load[t] < load[k]) k = t;
      load[k] += j.ms;
      if (!used[k]) {
        HIPCHK(hipStreamWaitEvent(ring[k], c->ev_fork, 0));
        used[k] = true;
      }
      const hipStream_t s = ring[k];
      if (j.q >= 0) {
        auto& W = c->work[j.q];
        set_gclass(ga, W);
        const int pk = c->profiling ? prof_begin(c, j.q, 1, s) : -1;
        ga.unit_threads = c->grad_unit_threads[j.q] ? c->grad_unit_threads[j.q] : 64;
        ga.gstat = c->d_gstat.p + 2 * j.q;
        if (c->grad_variant[j.q]) qc[j.q].coop_grad(ga, s);
        else qc[j.q].grad(ga, s);
        ga.gstat = nullptr;
        if (pk >= 0) prof_end(c, pk, s);
        W.grad_launches++;
      } else {
        int la, lb;
        pc_l(-1 - j.q, la, lb);
        launch_grad1e(la, lb, g1[-1 - j.q], s);
      }
    }
    for (int k = 1; k < kNs; ++k) {
      if (!used[k]) continue;
      HIPCHK(hipEventRecord(c->ev_join[k - 1], ring[k]));
      HIPCHK(hipStreamWaitEvent(st, c->ev_join[k - 1], 0));
    }
    HIPCHK(hipGetLastError());
    if (with_xc) xc_gradient(c, c->P.p, c->d_grad.p);
    std::vector<double> g(3 * c->total_atoms), gs(2 * kNumQuartetClasses);
    HIPCHK(hipMemcpyAsync(g.data(), c->d_grad.p, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(gs.data(), c->d_gstat.p, gs.size() * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    sync(c);
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      c->work[q].grad_quart += gs[2 * q];
      c->work[q].grad_primq += gs[2 * q + 1];
    }
    for (size_t k = 0; k < g.size(); ++k) Fout[k] = -g[k];
    if (c->md.on && c->md.synced) c->md.have_force = true;
    c->t_grad_ms += now_ms() - t0;
}
}  // namespace

bscf_status bscf_forces(bscf_ctx* c, double* Fout) {
  return guard([&] {
    need(c && Fout, BSCF_E_INVALID, "NULL argument");
    need(c->have_scf, BSCF_E_STATE, "forces need an SCF at the current geometry");
    HIPCHK(hipSetDevice(c->device));
    forces_impl(c, Fout, c->scf_xc);
  });
}

bscf_status bscf_forces_at(bscf_ctx* c, const double* P, const double* F, double* Fout,
                           double tau, int device_ptrs) {
  return guard([&] {
    need(c && P && F && Fout, BSCF_E_INVALID, "NULL argument");
    need(std::isfinite(tau), BSCF_E_INVALID, "bad Schwarz cutoff");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    // the screened work lists of the current geometry at this cutoff
    ensure_work(c, tau, c->split_tol, false);
    c->have_scf = false;   // the SCF density is replaced: forces need a new SCF
    const auto kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(c->P.p, P, c->mtot * sizeof(double), kind, c->stream));
    HIPCHK(hipMemcpyAsync(c->F.p, F, c->mtot * sizeof(double), kind, c->stream));
    forces_impl(c, Fout, c->xc != 0);
  });
}

// ------------------------------------------------------------ ring polymer

namespace {
constexpr double kKbHartreePerK = 3.166811563e-6;   // CODATA 2018

PimdArgs pimd_args(bscf_ctx* c) {
  auto& m = c->md;
  PimdArgs a;
  a.P = m.P;
  a.ncol = 3 * m.N;
  a.dt = m.o.dt;
  a.x = m.x.p;
  a.p = m.p.p;
  a.C = m.C.p;
  a.w = m.w.p;
  a.c1 = m.c1.p;
  a.c2 = m.c2.p;
  a.mass = m.mass.p;
  a.sig = m.sig.p;
  a.seed = m.o.seed;
  return a;
}

// forces of a half-step: the caller's [P][N][3] (host), or the context's
// last gradient at the current positions (sign -1)
const double* pimd_forces(bscf_ctx* c, const double* F, double& sign) {
  auto& m = c->md;
  if (F) {
    const size_t n = (size_t)m.P * 3 * m.N;
    for (size_t k = 0; k < n; ++k) need(std::isfinite(F[k]), BSCF_E_INVALID, "non-finite force");
    m.F.resize(n);
    HIPCHK(hipMemcpyAsync(m.F.p, F, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    sign = 1.0;
    return m.F.p;
  }
  need(m.have_force, BSCF_E_STATE, "no forces at the current ring-polymer positions");
  sign = -1.0;
  return c->d_grad.p;
}

void pimd_begin_impl(bscf_ctx* c, const double* F) {
  auto& m = c->md;
  double sign = 1.0;
  const double* f = pimd_forces(c, F, sign);
  const PimdArgs a = pimd_args(c);
  launch_pimd_ob(a, f, sign, m.o.thermostat, 2 * m.step, 0, c->stream);
  launch_pimd_a(a, c->stream);
  HIPCHK(hipGetLastError());
  m.synced = m.have_force = false;
}

void pimd_end_impl(bscf_ctx* c, const double* F) {
  auto& m = c->md;
  double sign = 1.0;
  const double* f = pimd_forces(c, F, sign);
  launch_pimd_ob(pimd_args(c), f, sign, m.o.thermostat, 2 * m.step + 1, 1, c->stream);
  HIPCHK(hipGetLastError());
  ++m.step;
}

void check_status(bscf_status rc) {
  if (rc != BSCF_OK) throw Error(rc, g_err);
}

// the context's geometry from the integrator's positions, then SCF and forces
void pimd_forces_here(bscf_ctx* c, const bscf_scf_opts* o, double* E, int* it, int* st,
                      double* Fout = nullptr) {
  auto& m = c->md;
  std::vector<double> x((size_t)m.P * 3 * m.N), F(x.size());
  HIPCHK(hipMemcpyAsync(x.data(), m.x.p, x.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  check_status(bscf_set_geometries(c, x.data()));
  m.synced = true;
  check_status(bscf_run_scf(c, o, E, it, st));
  forces_impl(c, F.data(), c->scf_xc);
  if (Fout) std::copy(F.begin(), F.end(), Fout);
}
}  // namespace

bscf_status bscf_pimd_default_opts(bscf_pimd_opts* o) {
  if (!o) return BSCF_E_INVALID;
  o->dt = 0.25 * 41.341373336;
  o->temperature = 300.0;
  o->thermostat = 1;
  o->tau_centroid = 100.0 * 41.341373336;
  o->friction_scale = 1.0;
  o->seed = 0;
  return BSCF_OK;
}

bscf_status bscf_pimd_init(bscf_ctx* c, const bscf_pimd_opts* opts, const double* masses,
                           const double* p0) {
  return guard([&] {
    need(c && opts && masses, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    const bscf_pimd_opts o = *opts;
    need(std::isfinite(o.dt) && o.dt > 0.0, BSCF_E_INVALID, "dt must be positive");
    need(std::isfinite(o.temperature) && o.temperature > 0.0, BSCF_E_INVALID,
         "temperature must be positive");
    need(o.thermostat == 0 || o.thermostat == 1, BSCF_E_INVALID, "thermostat must be 0 or 1");
    need(std::isfinite(o.friction_scale) && o.friction_scale > 0.0, BSCF_E_INVALID,
         "friction_scale must be positive");
    need(std::isfinite(o.tau_centroid), BSCF_E_INVALID, "bad tau_centroid");
    const int P = c->ninst, N = c->natoms[0];
    need(P <= kPimdMaxBeads, BSCF_E_UNSUPPORTED,
         "at most " + std::to_string(kPimdMaxBeads) + " beads");
    for (int i = 0; i < P; ++i) {
      need(c->natoms[i] == N, BSCF_E_INVALID, "beads must be copies of one system");
      for (int a = 0; a < N; ++a)
        need(c->Zs[c->atom_off[i] + a] == c->Zs[a], BSCF_E_INVALID, "beads must be copies of one system");
    }
    for (int a = 0; a < N; ++a)
      need(std::isfinite(masses[a]) && masses[a] > 0.0, BSCF_E_INVALID, "masses must be positive");
    const size_t n = (size_t)P * 3 * N;
    if (p0)
      for (size_t k = 0; k < n; ++k) need(std::isfinite(p0[k]), BSCF_E_INVALID, "non-finite momentum");
    HIPCHK(hipSetDevice(c->device));
    // normal modes of the cyclic chain, their frequencies and the O-step
    // factors (host, FP64)
    const double kT = kKbHartreePerK * o.temperature;
    const double wp = std::sqrt((double)P) * kT;
    std::vector<double> C((size_t)P * P), w(P), c1(P), c2(P), sig(N), mass(masses, masses + N);
    for (int j = 0; j < P; ++j)
      for (int k = 0; k < P; ++k) {
        double v;
        if (k == 0) v = 1.0 / std::sqrt((double)P);
        else if (2 * k < P) v = std::sqrt(2.0 / P) * std::cos(2.0 * M_PI * j * k / P);
        else if (2 * k == P) v = (j % 2 ? -1.0 : 1.0) / std::sqrt((double)P);
        else v = std::sqrt(2.0 / P) * std::sin(2.0 * M_PI * j * k / P);
        C[(size_t)j * P + k] = v;
      }
    for (int k = 0; k < P; ++k) {
      w[k] = 2.0 * wp * std::sin(k * M_PI / P);
      const double gam = k == 0 ? (o.tau_centroid > 0.0 ? 1.0 / o.tau_centroid : 0.0)
                                : 2.0 * o.friction_scale * w[k];
      c1[k] = std::exp(-0.5 * gam * o.dt);
      c2[k] = std::sqrt(1.0 - c1[k] * c1[k]);
    }
    for (int a = 0; a < N; ++a) sig[a] = std::sqrt(mass[a] * kT);
    auto& m = c->md;
    m.on = false;
    const hipStream_t s = c->stream;
    m.C.upload(C, s);
    m.w.upload(w, s);
    m.c1.upload(c1, s);
    m.c2.upload(c2, s);
    m.sig.upload(sig, s);
    m.mass.upload(mass, s);
    m.x.upload(c->xyz, s);
    std::vector<double> pv(n, 0.0);
    if (p0) pv.assign(p0, p0 + n);
    m.p.upload(pv, s);
    m.F.resize(n);
    sync(c);
    m.P = P;
    m.N = N;
    m.o = o;
    m.step = 0;
    m.on = true;
    m.synced = true;
    m.have_force = false;
  });
}

bscf_status bscf_pimd_begin(bscf_ctx* c, const double* forces) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->md.on, BSCF_E_STATE, "no ring polymer: call bscf_pimd_init");
    HIPCHK(hipSetDevice(c->device));
    pimd_begin_impl(c, forces);
    sync(c);
  });
}

bscf_status bscf_pimd_end(bscf_ctx* c, const double* forces) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->md.on, BSCF_E_STATE, "no ring polymer: call bscf_pimd_init");
    HIPCHK(hipSetDevice(c->device));
    pimd_end_impl(c, forces);
    sync(c);
  });
}

bscf_status bscf_pimd_step(bscf_ctx* c, const bscf_scf_opts* opts, double* E, int* n_iter,
                           int* status, double* forces) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->md.on, BSCF_E_STATE, "no ring polymer: call bscf_pimd_init");
    HIPCHK(hipSetDevice(c->device));
    if (!c->md.have_force) pimd_forces_here(c, opts, nullptr, nullptr, nullptr);
    pimd_begin_impl(c, nullptr);
    pimd_forces_here(c, opts, E, n_iter, status, forces);
    pimd_end_impl(c, nullptr);
    sync(c);
  });
}

bscf_status bscf_pimd_state(bscf_ctx* c, double* x, double* p, double* obs) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->md.on, BSCF_E_STATE, "no ring polymer: call bscf_pimd_init");
    HIPCHK(hipSetDevice(c->device));
    auto& m = c->md;
    const size_t n = (size_t)m.P * 3 * m.N;
    std::vector<double> hx(n), hp(n);
    HIPCHK(hipMemcpyAsync(hx.data(), m.x.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hp.data(), m.p.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (x) std::copy(hx.begin(), hx.end(), x);
    if (p) std::copy(hp.begin(), hp.end(), p);
    if (obs) {
      std::vector<double> mass(m.N);
      HIPCHK(hipMemcpy(mass.data(), m.mass.p, m.N * sizeof(double), hipMemcpyDeviceToHost));
      const double wp = std::sqrt((double)m.P) * kKbHartreePerK * m.o.temperature;
      double ke = 0.0, sp = 0.0;
      for (int j = 0; j < m.P; ++j)
        for (int a = 0; a < m.N; ++a)
          for (int d = 0; d < 3; ++d) {
            const size_t i = ((size_t)j * m.N + a) * 3 + d;
            const size_t i1 = ((size_t)((j + 1) % m.P) * m.N + a) * 3 + d;
            ke += hp[i] * hp[i] / (2.0 * mass[a]);
            const double dx = hx[i] - hx[i1];
            sp += 0.5 * mass[a] * wp * wp * dx * dx;
          }
      obs[0] = ke;
      obs[1] = sp;
      obs[2] = (double)m.step;
    }
  });
}

// ------------------------------------------------------------ string method

namespace {
// all instances copies of instance 0's composition
void require_copies(bscf_ctx* c, const char* what) {
  const int N = c->natoms[0];
  for (int i = 0; i < c->ninst; ++i) {
    need(c->natoms[i] == N, BSCF_E_INVALID, what);
    for (int a = 0; a < N; ++a)
      need(c->Zs[c->atom_off[i] + a] == c->Zs[a], BSCF_E_INVALID, what);
  }
}

// evolve with forces (caller's host array, or sign -1 on the context's
// gradient), then reparametrise into the image buffer
void string_update(bscf_ctx* c, const double* F, double sign) {
  auto& g = c->str;
  const int ncol = 3 * g.N;
  launch_string_evolve(g.n, ncol, g.x.p, F, sign, g.o.step, g.o.fix_ends, c->stream);
  launch_string_reparam(g.n, ncol, g.x.p, g.xt.p, g.arc.p, c->stream);
  HIPCHK(hipGetLastError());
  std::swap(g.x.p, g.xt.p);
  g.synced = false;
  ++g.iters;
}
}  // namespace

bscf_status bscf_string_default_opts(bscf_string_opts* o) {
  if (!o) return BSCF_E_INVALID;
  o->step = 0.5;
  o->fix_ends = 0;
  return BSCF_OK;
}

bscf_status bscf_string_init(bscf_ctx* c, const bscf_string_opts* opts) {
  return guard([&] {
    need(c && opts, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    need(std::isfinite(opts->step) && opts->step > 0.0, BSCF_E_INVALID, "step must be positive");
    need(opts->fix_ends == 0 || opts->fix_ends == 1, BSCF_E_INVALID, "fix_ends must be 0 or 1");
    need(c->ninst >= 2, BSCF_E_INVALID, "a string needs at least two images");
    need(c->ninst <= kStringMaxImages, BSCF_E_UNSUPPORTED,
         "at most " + std::to_string(kStringMaxImages) + " images");
    require_copies(c, "images must be copies of one system");
    HIPCHK(hipSetDevice(c->device));
    auto& g = c->str;
    g.on = false;
    const size_t n = (size_t)c->ninst * 3 * c->natoms[0];
    g.x.upload(c->xyz, c->stream);
    g.xt.resize(n);
    g.F.resize(n);
    g.arc.resize(c->ninst);
    sync(c);
    g.n = c->ninst;
    g.N = c->natoms[0];
    g.o = *opts;
    g.iters = 0;
    g.synced = true;
    g.on = true;
  });
}

bscf_status bscf_string_step(bscf_ctx* c, const bscf_scf_opts* opts, double* E, int* n_iter,
                             int* status, double* forces) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->str.on, BSCF_E_STATE, "no string: call bscf_string_init");
    HIPCHK(hipSetDevice(c->device));
    auto& g = c->str;
    std::vector<double> x((size_t)g.n * 3 * g.N);
    if (!g.synced) {
      HIPCHK(hipMemcpyAsync(x.data(), g.x.p, x.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
      sync(c);
      check_status(bscf_set_geometries(c, x.data()));
      g.synced = true;
    }
    check_status(bscf_run_scf(c, opts, E, n_iter, status));
    forces_impl(c, x.data(), c->scf_xc);
    if (forces) std::copy(x.begin(), x.end(), forces);
    string_update(c, c->d_grad.p, -1.0);
    sync(c);
  });
}

bscf_status bscf_string_evolve(bscf_ctx* c, const double* forces) {
  return guard([&] {
    need(c && forces, BSCF_E_INVALID, "NULL argument");
    need(c->str.on, BSCF_E_STATE, "no string: call bscf_string_init");
    HIPCHK(hipSetDevice(c->device));
    auto& g = c->str;
    const size_t n = (size_t)g.n * 3 * g.N;
    for (size_t k = 0; k < n; ++k) need(std::isfinite(forces[k]), BSCF_E_INVALID, "non-finite force");
    HIPCHK(hipMemcpyAsync(g.F.p, forces, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    string_update(c, g.F.p, 1.0);
    sync(c);
  });
}

bscf_status bscf_string_state(bscf_ctx* c, double* x, double* arc) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(c->str.on, BSCF_E_STATE, "no string: call bscf_string_init");
    HIPCHK(hipSetDevice(c->device));
    auto& g = c->str;
    if (x)
      HIPCHK(hipMemcpyAsync(x, g.x.p, (size_t)g.n * 3 * g.N * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    if (arc) {   // the arc positions of the current images (the redistribution is discarded)
      launch_string_reparam(g.n, 3 * g.N, g.x.p, g.xt.p, g.arc.p, c->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(arc, g.arc.p, g.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    sync(c);
  });
}

bscf_status bscf_get_density(bscf_ctx* c, int inst, double* P, int device_ptr) {
  return guard([&] {
    need(c && P && inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "bad arguments");
    const size_t nn = (size_t)c->nbf[inst] * c->nbf[inst];
    HIPCHK(hipMemcpyAsync(P, c->P.p + c->moff[inst], nn * sizeof(double),
                          device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

bscf_status bscf_get_one_electron(bscf_ctx* c, int inst, double* S, double* H) {
  return guard([&] {
    need(c && inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "bad arguments");
    require_geom(c);
    const size_t nn = (size_t)c->nbf[inst] * c->nbf[inst];
    if (S) HIPCHK(hipMemcpyAsync(S, c->S.p + c->moff[inst], nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (H) HIPCHK(hipMemcpyAsync(H, c->H.p + c->moff[inst], nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

bscf_status bscf_eri_tensor(bscf_ctx* c, int inst, double* out) {
  return guard([&] {
    need(c && out && inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "bad arguments");
    require_geom(c);
    const int n = c->nbf[inst];
    need(n <= 64, BSCF_E_INVALID, "eri_tensor is limited to n <= 64");
    const size_t n4 = (size_t)n * n * n * n;
    DevBuf<double> d_out;
    d_out.resize(n4);
    launch_fill(d_out.p, (long long)n4, 0.0, c->stream);
    const QuartetClass* qc = quartet_classes();
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      const int X = pclass(qc[q].la, qc[q].lb), Y = pclass(qc[q].lc, qc[q].ld);
      std::vector<int> quart;
      std::vector<int> bl, kl;
      for (int pid : c->pairs_by_class[X])
        if (c->shells[c->pairs[pid].a].inst == inst) bl.push_back(pid);
      for (int pid : c->pairs_by_class[Y])
        if (c->shells[c->pairs[pid].a].inst == inst) kl.push_back(pid);
      for (int b : bl)
        for (int k : kl) {
          if (X == Y && k > b) continue;
          quart.push_back(b);
          quart.push_back(k);
        }
      if (quart.empty()) continue;
      DevBuf<int> dq;
      dq.upload(quart, c->stream);
      TensorArgs ta{dq.p, (int)quart.size() / 2, c->d_pairs.p, c->d_prims.p, c->d_shells.p,
                    c->d_boys64.p, n, d_out.p};
      qc[q].tensor(ta, c->stream);
      sync(c);
    }
    HIPCHK(hipMemcpyAsync(out, d_out.p, n4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

bscf_status bscf_schwarz(bscf_ctx* c, int inst, double* Qout, int nsh) {
  return guard([&] {
    need(c && Qout && inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "bad arguments");
    require_geom(c);
    need(nsh == c->nshell[inst], BSCF_E_INVALID, "nsh does not match the instance");
    const int s0 = c->shell_off[inst];
    for (size_t p = 0; p < c->pairs.size(); ++p) {
      const ShellPair& sp = c->pairs[p];
      if (c->shells[sp.a].inst != inst) continue;
      const int a = sp.a - s0, b = sp.b - s0;
      Qout[a * nsh + b] = Qout[b * nsh + a] = c->Q[p];
    }
  });
}

bscf_status bscf_instance_info(bscf_ctx* c, int inst, int* nbf, int* nshell, int* natom) {
  return guard([&] {
    need(c && inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "bad arguments");
    if (nbf) *nbf = c->nbf[inst];
    if (nshell) *nshell = c->nshell[inst];
    if (natom) *natom = c->natoms[inst];
  });
}

bscf_status bscf_work_counts(bscf_ctx* c, double* nq, double* npq, double* flops) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    require_geom(c);
    join_work(c);
    if (c->work_tau < 0) ensure_work(c, 1e-12, c->split_tol, false);
    const QuartetClass* qc = quartet_classes();
    double a = 0, b = 0, f = 0;
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      a += c->work[q].nquart;
      b += c->work[q].nprimq;
      const int nout = ncart(qc[q].la) * ncart(qc[q].lb) * ncart(qc[q].lc) * ncart(qc[q].ld);
      // per primitive quartet: setup, Boys and VRR as counted from the code by
      // the generator; per contracted quartet: HRR + digestion (6 FMAs = 12
      // FLOP per integral)
      f += c->work[q].nprimq * qc[q].prim_flops + c->work[q].nquart * (qc[q].hrr_flops + 12.0 * nout);
    }
    if (nq) *nq = a;
    if (npq) *npq = b;
    if (flops) *flops = f;
  });
}

bscf_status bscf_set_deterministic(bscf_ctx* c, int on) {
  return guard([&] {
    need(c != nullptr && (on == 0 || on == 1), BSCF_E_INVALID, "bad arguments");
    c->det = on == 1;
  });
}

bscf_status bscf_set_xc(bscf_ctx* c, int functional) {
  return guard([&] {
    need(c != nullptr && (functional == BSCF_XC_NONE || functional == BSCF_XC_B3LYP),
         BSCF_E_INVALID, "bad arguments");
    c->xc = functional;
  });
}

bscf_status bscf_xc_matrix(bscf_ctx* c, const double* P, double* Vxc, double* Exc,
                           int device_ptrs) {
  return guard([&] {
    need(c && P && Vxc && Exc, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    const auto kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    c->have_scf = false;   // the SCF density is replaced: forces need a new SCF
    HIPCHK(hipMemcpyAsync(c->P.p, P, c->mtot * sizeof(double), kind, c->stream));
    xc_build(c, c->P.p, false);
    const auto back = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(Vxc, c->xcs.V.p, c->mtot * sizeof(double), back, c->stream));
    HIPCHK(hipMemcpyAsync(Exc, c->xcs.exc.p, c->ninst * sizeof(double), back, c->stream));
    sync(c);
  });
}

bscf_status bscf_xc_grid_size(bscf_ctx* c, int inst, long long* npts) {
  return guard([&] {
    need(c && npts, BSCF_E_INVALID, "NULL argument");
    need(inst >= 0 && inst < c->ninst, BSCF_E_INVALID, "instance out of range");
    *npts = (long long)c->natoms[inst] * kXcPerAtom;
  });
}

bscf_status bscf_xc_functional(bscf_ctx* c, int n, const double* rho, const double* sigma,
                               double* e, double* vrho, double* vsigma) {
  return guard([&] {
    need(c && n >= 0, BSCF_E_INVALID, "bad arguments");
    if (n == 0) return;
    need(rho && sigma && e && vrho && vsigma, BSCF_E_INVALID, "NULL argument");
    HIPCHK(hipSetDevice(c->device));
    DevBuf<double> d;
    d.resize((size_t)5 * n);
    const hipStream_t st = c->stream;
    HIPCHK(hipMemcpyAsync(d.p, rho, n * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.p + n, sigma, n * sizeof(double), hipMemcpyHostToDevice, st));
    launch_xc_functional(n, d.p, d.p + n, d.p + 2 * n, d.p + 3 * n, d.p + 4 * n, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(e, d.p + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(vrho, d.p + 3 * n, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(vsigma, d.p + 4 * n, n * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
  });
}

bscf_status bscf_set_profiling(bscf_ctx* c, int on) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    c->profiling = on != 0;
  });
}

bscf_status bscf_reset_stats(bscf_ctx* c) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    join_work(c);
    prof_collect(c);
    collect_kept(c);
    for (auto& W : c->work) {
      W.done_quart = W.done_primq = W.kernel_ms = W.grad_ms = W.done_quart32 = 0;
      W.grad_quart = W.grad_primq = 0;
      W.screened_quart = 0;
      W.launches = W.grad_launches = 0;
    }
    c->t_fock_ms = c->t_scf_ms = c->t_grad_ms = c->t_setup_ms = c->t_fock_gpu_ms = c->t_work_ms = 0;
    c->t_work_host_ms = 0;
    c->t_work_phase_ms[0] = c->t_work_phase_ms[1] = c->t_work_phase_ms[2] = 0;
    c->fock_builds = c->scf_iters = 0;
    c->sp2_calls = c->sp2_steps = c->sp2_needed = c->sp2_fallbacks = 0;
    c->inc_builds = 0;
    c->graph_launches = c->graph_captures = 0;
    c->fock_graph_launches = c->fock_graph_captures = c->graph_memset_nodes = 0;
    for (int k = 0; k < 7; ++k) {
      c->xc_ms[k] = 0;
      c->xc_launches[k] = 0;
    }
    c->xc_builds = 0;
    c->xc_points = c->xc_gemm_flops = c->xc_basis_bytes = c->xc_point_bytes = 0;
  });
}

bscf_status bscf_get_stats(bscf_ctx* c, char* buf, int len) {
  return guard([&] {
    need(c && buf && len > 0, BSCF_E_INVALID, "bad arguments");
    join_work(c);
    prof_collect(c);
    collect_kept(c);
    std::ostringstream s;
    s << "{\"fock_builds\": " << c->fock_builds << ", \"scf_iterations\": " << c->scf_iters
      << ", \"t_fock_ms\": " << c->t_fock_ms << ", \"t_scf_ms\": " << c->t_scf_ms
      << ", \"t_grad_ms\": " << c->t_grad_ms << ", \"t_setup_ms\": " << c->t_setup_ms
      << ", \"t_fock_gpu_ms\": " << c->t_fock_gpu_ms << ", \"t_work_ms\": " << c->t_work_ms
      << ", \"t_work_host_ms\": " << c->t_work_host_ms << ", \"t_work_phase_ms\": ["
      << c->t_work_phase_ms[0] << ", " << c->t_work_phase_ms[1] << ", " << c->t_work_phase_ms[2] << "]"
      << ", \"sp2_calls\": " << c->sp2_calls << ", \"sp2_steps\": " << c->sp2_steps
      << ", \"sp2_steps_needed\": " << c->sp2_needed
      << ", \"sp2_fallbacks\": " << c->sp2_fallbacks << ", \"incremental_builds\": " << c->inc_builds
      << ", \"graph_launches\": " << c->graph_launches << ", \"graph_captures\": " << c->graph_captures
      << ", \"fock_graph_launches\": " << c->fock_graph_launches
      << ", \"fock_graph_captures\": " << c->fock_graph_captures
      << ", \"graph_memset_nodes\": " << c->graph_memset_nodes
      << ", \"xc\": {\"builds\": " << c->xc_builds << ", \"points\": " << c->xc_points
      << ", \"gemm_flops\": " << c->xc_gemm_flops << ", \"basis_bytes\": " << c->xc_basis_bytes
      << ", \"point_bytes\": " << c->xc_point_bytes << ", \"ms\": {";
    const char* xn[7] = {"basis", "gemm", "point", "gemm_v", "build", "grad_basis_term",
                         "grad_weight_term"};
    for (int k = 0; k < 7; ++k)
      s << (k ? ", " : "") << "\"" << xn[k] << "\": [" << c->xc_ms[k] << ", " << c->xc_launches[k] << "]";
    s << "}}, \"classes\": {";
    const QuartetClass* qc = quartet_classes();
    for (int q = 0; q < kNumQuartetClasses; ++q) {
      const auto& W = c->work[q];
      const double nout = ncart(qc[q].la) * ncart(qc[q].lb) * ncart(qc[q].lc) * ncart(qc[q].ld);
      const double flops = W.done_primq * qc[q].prim_flops + W.done_quart * (qc[q].hrr_flops + 12.0 * nout);
      s << (q ? ", " : "") << "\"" << qc[q].la << qc[q].lb << qc[q].lc << qc[q].ld
        << "\": {\"quartets\": " << W.nquart << ", \"prim_quartets\": " << W.nprimq
        << ", \"quartets_fp32_list\": " << W.nquart32 << ", \"done_quartets_fp32\": " << W.done_quart32
        << ", \"items\": " << W.items.size() << ", \"done_quartets\": " << W.done_quart
        << ", \"done_prim_quartets\": " << W.done_primq << ", \"done_flops\": " << flops
        << ", \"screened_quartets_built\": " << W.screened_quart
        << ", \"prim_flops\": " << qc[q].prim_flops << ", \"hrr_flops\": " << qc[q].hrr_flops
        << ", \"kernel_ms\": " << W.kernel_ms << ", \"launches\": " << W.launches
        << ", \"grad_ms\": " << W.grad_ms << ", \"grad_launches\": " << W.grad_launches
        << ", \"grad_quartets\": " << W.grad_quart << ", \"grad_prim_quartets\": " << W.grad_primq
        << ", \"grad_flops\": "
        << W.grad_primq * qc[q].grad_prim_flops + W.grad_quart * qc[q].grad_con_flops
        << ", \"private_bytes\": [" << c->private_bytes[q][0] << ", " << c->private_bytes[q][1]
        << ", " << c->private_bytes[q][2] << "], \"variant\": [" << c->fock_variant[0][q] << ", "
        << c->fock_variant[1][q] << ", " << c->grad_variant[q] << "], \"tune_ms\": ["
        << c->tune_ms[0][q][0] << ", " << c->tune_ms[0][q][1] << ", " << c->tune_grad_ms[q][0]
        << ", " << c->tune_grad_ms[q][1] << "], \"tune_ms_mixed\": [" << c->tune_ms[1][q][0] << ", "
        << c->tune_ms[1][q][1] << ", " << c->tune_ms[1][q][2] << "]}";
    }
    s << "}}";
    const std::string str = s.str();
    need((int)str.size() < len, BSCF_E_INVALID, "buffer too small");
    memcpy(buf, str.c_str(), str.size() + 1);
  });
}

double bscf_boys_table_entry(int m, int k) {
  static std::vector<double> tab;
  if (tab.empty()) {
    tab.resize(kBoysRows * kBoysCols);
    boys_table_host(tab.data());
  }
  if (m < 0 || m >= kBoysCols || k < 0 || k >= kBoysRows) return NAN;
  return tab[k * kBoysCols + m];
}

bscf_status bscf_boys(bscf_ctx* c, int m_max, int n, const double* T, double* out, int precision) {
  return guard([&] {
    need(c && T && out && n > 0 && m_max >= 0 && m_max <= 12, BSCF_E_INVALID, "bad arguments");
    DevBuf<double> dT, dO;
    std::vector<double> t(T, T + n);
    dT.upload(t, c->stream);
    dO.resize((size_t)n * (m_max + 1));
    launch_boys_eval(m_max, n, dT.p, dO.p, precision, c->d_boys64.p, c->d_boys32.p, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, dO.p, (size_t)n * (m_max + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

bscf_status bscf_guess_train(bscf_ctx* c, int n_adam_steps, float* loss) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    need(n_adam_steps >= 0, BSCF_E_INVALID, "negative step count");
    HIPCHK(hipSetDevice(c->device));
    const float l = c->guess.train(n_adam_steps, c->stream);
    if (loss) *loss = l;
  });
}

bscf_status bscf_guess_configure(bscf_ctx* c, int din, int dout, unsigned seed) {
  return guard([&] {
    need(c != nullptr && din > 0 && dout > 0, BSCF_E_INVALID, "bad arguments");
    HIPCHK(hipSetDevice(c->device));
    c->guess.configure_detached(din, dout, seed);
  });
}

bscf_status bscf_guess_param_count(bscf_ctx* c, int* din, int* dout, long* n) {
  return guard([&] {
    need(c != nullptr, BSCF_E_INVALID, "NULL context");
    if (din) *din = c->guess.din();
    if (dout) *dout = c->guess.dout();
    if (n) *n = c->guess.din() ? c->guess.nparams() : 0;
  });
}

bscf_status bscf_guess_set_params(bscf_ctx* c, const float* params, long n) {
  return guard([&] {
    need(c && params, BSCF_E_INVALID, "NULL argument");
    need(c->guess.din() > 0, BSCF_E_STATE, "network not configured");
    HIPCHK(hipSetDevice(c->device));
    c->guess.set_params(params, n, c->stream);
  });
}

bscf_status bscf_guess_get_params(bscf_ctx* c, float* params, long n) {
  return guard([&] {
    need(c && params, BSCF_E_INVALID, "NULL argument");
    need(c->guess.din() > 0, BSCF_E_STATE, "network not configured");
    HIPCHK(hipSetDevice(c->device));
    c->guess.get_params(params, n, c->stream);
  });
}

bscf_status bscf_guess_eval(bscf_ctx* c, int rows, const float* X, const float* T, const float* mask,
                            float* Y, float* grad, float* loss) {
  return guard([&] {
    need(c && X && rows > 0, BSCF_E_INVALID, "bad arguments");
    need((T == nullptr) == (mask == nullptr), BSCF_E_INVALID, "targets and mask go together");
    need(c->guess.din() > 0, BSCF_E_STATE, "network not configured");
    HIPCHK(hipSetDevice(c->device));
    c->guess.eval_rows(rows, X, T, mask, Y, grad, loss, c->stream);
  });
}

bscf_status bscf_guess_eval_noalloc(bscf_ctx* c, int rows, const float* X, float* Y) {
  return guard([&] {
    need(c && X && Y, BSCF_E_INVALID, "NULL argument");
    need(rows > 0 && rows <= mlp::kNoAllocRows, BSCF_E_INVALID,
         "rows must be 1.." + std::to_string(mlp::kNoAllocRows) + " for the allocation-free evaluation");
    need(c->guess.din() > 0, BSCF_E_STATE, "network not configured");
    HIPCHK(hipSetDevice(c->device));
    c->guess.eval_noalloc(c->device, rows, X, Y, c->stream);
  });
}

bscf_status bscf_guess_fit(bscf_ctx* c, int rows, const float* X, const float* T, const float* mask,
                           int steps, float lr, float* loss) {
  return guard([&] {
    need(c && X && T && mask && rows > 0 && steps > 0 && lr > 0.f, BSCF_E_INVALID, "bad arguments");
    need(c->guess.din() > 0, BSCF_E_STATE, "network not configured");
    HIPCHK(hipSetDevice(c->device));
    const float l = c->guess.fit_rows(rows, X, T, mask, steps, lr, c->stream);
    if (loss) *loss = l;
  });
}

}  // extern "C"

namespace {
constexpr int kCkptMagic = 0x4B435342;   // "BSCK"
constexpr int kCkptVersion = 2;

template <typename T>
void put(std::ostream& f, const T& v) {
  f.write(reinterpret_cast<const char*>(&v), sizeof(T));
}
template <typename T>
void put(std::ostream& f, const std::vector<T>& v) {
  f.write(reinterpret_cast<const char*>(v.data()), v.size() * sizeof(T));
}
template <typename T>
T get(std::istream& f) {
  T v{};
  f.read(reinterpret_cast<char*>(&v), sizeof(T));
  need(bool(f), BSCF_E_INVALID, "checkpoint: truncated file");
  return v;
}
template <typename T>
std::vector<T> get(std::istream& f, size_t n) {
  std::vector<T> v(n);
  f.read(reinterpret_cast<char*>(v.data()), n * sizeof(T));
  need(bool(f), BSCF_E_INVALID, "checkpoint: truncated file");
  return v;
}
template <typename T>
std::vector<T> fetch(bscf_ctx* c, const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  return h;
}
}  // namespace

extern "C" {

bscf_status bscf_checkpoint_save(bscf_ctx* c, const char* path) {
  return guard([&] {
    need(c && path, BSCF_E_INVALID, "NULL argument");
    require_geom(c);
    HIPCHK(hipSetDevice(c->device));
    const int ni = c->ninst, na = c->total_atoms;
    const size_t mt = (size_t)c->mtot;
    const auto P = fetch(c, c->P.p, mt), C1 = fetch(c, c->Cacc.p, mt), C2 = fetch(c, c->Cprev.p, mt);
    auto& m = c->md;
    const size_t nx = (size_t)m.P * 3 * m.N;
    std::vector<double> mx, mp, mmass, grad;
    if (m.on) {
      mx = fetch(c, m.x.p, nx);
      mp = fetch(c, m.p.p, nx);
      mmass = fetch(c, m.mass.p, (size_t)m.N);
      if (m.have_force) grad = fetch(c, c->d_grad.p, (size_t)3 * na);
    }
    sync(c);
    std::ofstream f(path, std::ios::binary);
    need(bool(f), BSCF_E_INVALID, std::string("checkpoint: cannot write ") + path);
    put(f, kCkptMagic);
    put(f, kCkptVersion);
    put(f, ni);
    put(f, na);
    put(f, c->mtot);
    put(f, c->natoms);
    put(f, c->Zs);
    put(f, c->charge);
    put(f, c->nbf);
    put(f, c->xyz);
    put(f, (int)c->have_C);
    put(f, c->h_ccount);
    put(f, P);
    put(f, C1);
    put(f, C2);
    put(f, (int)m.on);
    if (m.on) {
      put(f, m.o.dt);
      put(f, m.o.temperature);
      put(f, m.o.thermostat);
      put(f, m.o.tau_centroid);
      put(f, m.o.friction_scale);
      put(f, m.o.seed);
      put(f, m.P);
      put(f, m.N);
      put(f, m.step);
      put(f, (int)m.synced);
      put(f, (int)m.have_force);
      put(f, mmass);
      put(f, mx);
      put(f, mp);
      if (m.have_force) put(f, grad);
    }
    const int net = c->guess.din() > 0 ? 1 : 0;
    put(f, net);
    if (net) {
      c->guess.save(f);
      c->guess.save_run(f, c->mtot);
    }
    f.flush();
    need(bool(f), BSCF_E_INVALID, std::string("checkpoint: write failed: ") + path);
  });
}

bscf_status bscf_checkpoint_load(bscf_ctx* c, const char* path) {
  return guard([&] {
    need(c && path, BSCF_E_INVALID, "NULL argument");
    need(c->ninst > 0, BSCF_E_INVALID, "set instances first");
    std::ifstream f(path, std::ios::binary);
    need(bool(f), BSCF_E_INVALID, std::string("checkpoint: cannot read ") + path);
    // everything is read and checked on the host before the context changes
    need(get<int>(f) == kCkptMagic && get<int>(f) == kCkptVersion, BSCF_E_INVALID,
         "checkpoint: not a checkpoint file of this version");
    const int ni = get<int>(f), na = get<int>(f);
    const long long mtot = get<long long>(f);
    need(ni == c->ninst && na == c->total_atoms && mtot == c->mtot, BSCF_E_INVALID,
         "checkpoint: a different batch");
    need(get<int>(f, ni) == c->natoms && get<int>(f, na) == c->Zs &&
             get<int>(f, ni) == c->charge && get<int>(f, ni) == c->nbf,
         BSCF_E_INVALID, "checkpoint: a different batch or basis");
    const auto xyz = get<double>(f, (size_t)3 * na);
    const int have_C = get<int>(f);
    const auto ccount = get<int>(f, ni);
    const size_t mt = (size_t)mtot;
    const auto P = get<double>(f, mt), C1 = get<double>(f, mt), C2 = get<double>(f, mt);
    const int md_on = get<int>(f);
    bscf_pimd_opts o{};
    int mP = 0, mN = 0, synced = 0, have_force = 0;
    uint64_t step = 0;
    std::vector<double> mmass, mx, mp, grad;
    if (md_on) {
      o.dt = get<double>(f);
      o.temperature = get<double>(f);
      o.thermostat = get<int>(f);
      o.tau_centroid = get<double>(f);
      o.friction_scale = get<double>(f);
      o.seed = get<unsigned long long>(f);
      mP = get<int>(f);
      mN = get<int>(f);
      step = get<uint64_t>(f);
      synced = get<int>(f);
      have_force = get<int>(f);
      need(mP == ni && mN == c->natoms[0], BSCF_E_INVALID, "checkpoint: a different ring polymer");
      const size_t nx = (size_t)mP * 3 * mN;
      mmass = get<double>(f, (size_t)mN);
      mx = get<double>(f, nx);
      mp = get<double>(f, nx);
      if (have_force) grad = get<double>(f, (size_t)3 * na);
    }
    const int net = get<int>(f);
    mlp::Guess::Saved model;
    mlp::Guess::RunState run;
    if (net) {
      model = mlp::Guess::read(f);
      run = mlp::Guess::read_run(f, model.din, model.dout);
      need(!run.have_prev || (long long)run.rprev.size() == c->mtot, BSCF_E_INVALID,
           "checkpoint: a different batch");
    }
    need(bool(f), BSCF_E_INVALID, "checkpoint: truncated file");
    // geometry (and with it S, H, the Schwarz bounds and the work lists), the
    // carried densities and orbitals, then the ring polymer at its saved
    // step, then the network
    check_status(bscf_set_geometries(c, xyz.data()));
    HIPCHK(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    c->P.upload(P, s);
    c->Cacc.upload(C1, s);
    c->Cprev.upload(C2, s);
    c->h_ccount = ccount;
    c->have_C = have_C != 0;
    if (md_on) {
      check_status(bscf_pimd_init(c, &o, mmass.data(), mp.data()));
      auto& m = c->md;
      m.x.upload(mx, s);
      m.step = step;
      m.synced = synced != 0;
      if (have_force) c->d_grad.upload(grad, s);
      m.have_force = have_force != 0;
    }
    if (net) {
      c->guess.apply(model);
      c->guess.apply_run(run, c->mtot);
    }
    sync(c);
  });
}

bscf_status bscf_guess_save(bscf_ctx* c, const char* path) {
  return guard([&] {
    need(c && path, BSCF_E_INVALID, "NULL argument");
    c->guess.save(path);
  });
}

bscf_status bscf_guess_load(bscf_ctx* c, const char* path) {
  return guard([&] {
    need(c && path, BSCF_E_INVALID, "NULL argument");
    c->guess.load(path);
  });
}

}  // extern "C"
