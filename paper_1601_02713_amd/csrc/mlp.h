// Learned SCF guess (mlp.hip): a two-hidden-layer perceptron over atom pairs
// that corrects the standard previous-step density guess of each instance.
//
// One row per atom pair (A, B) of an instance with |R_AB| <= kCutoff (A = B
// included), the lower (Z, index) atom first.  Inputs: the element-pair
// one-hot, R_AB and |R_AB|, the displacements of A and B since the previous
// step, the P_AB block of the standard guess and the block of the previous
// step's residual (converged minus standard guess), blocks padded to
// bmax x bmax with bmax the largest per-atom basis size.  Output: the residual
// block of this step; the last input block (the previous residual) is added to
// the output (a residual connection), so an untrained network extrapolates the
// residual and training learns the correction.  The guess is the standard
// guess plus the prediction
// (diagonal blocks symmetrised), checked for finite values and a bounded size,
// otherwise the standard guess stands (status BSCF_FALLBACK_USED).
//
// Training data are recorded after every converged SCF that started from the
// standard guess; training is full-batch Adam on the last kReplaySteps
// recorded steps, with the project's own FP32 kernels: an MFMA GEMM with a
// fused bias/ReLU epilogue, the masked squared-error gradient, ReLU masks,
// column sums and the Adam update.
#pragma once
#include <hip/hip_runtime.h>

#include <iosfwd>
#include <string>
#include <vector>

namespace bscf {
namespace mlp {

constexpr int kHidden = 256;
constexpr int kReplaySteps = 4;
constexpr double kCutoff = 8.0;       // bohr
constexpr int kGeoFeatures = 10;      // R_AB (3), |R_AB|, dA (3), dB (3)

// Host view of the batch the engine hands over.
struct Batch {
  int ninst = 0;
  const long long* moff = nullptr;     // per instance, host
  const int* nbf = nullptr;            // per instance, host
  const int* natoms = nullptr;         // per instance, host
  const int* atom_off = nullptr;       // per instance, host
  const int* Z = nullptr;              // per global atom, host
  const double* xyz = nullptr;         // per global atom, bohr, host
  const int* atom_bf0 = nullptr;       // per global atom: first basis function in its instance
  const int* atom_nbf = nullptr;       // per global atom: basis functions on it
  int total_atoms = 0;
  size_t mtot = 0;                     // elements of all per-instance matrices
  double* P = nullptr;                 // device density (the guess is written here)
  hipStream_t stream = nullptr;
  size_t xyz_len() const { return 3 * (size_t)total_atoms; }
};

template <typename T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf();
  void resize(size_t m);   // contents undefined after growth
};

// Largest row count of the allocation-free evaluation (its hidden activations
// sit in a fixed per-GPU array of 2 x kNoAllocRows x kHidden floats, 16 MiB).
constexpr int kNoAllocRows = 8192;
// Finds the device address of that array on `device` (which must be current)
// once per device; called by context creation.
void init_noalloc_scratch(int device);

class Guess {
 public:
  ~Guess();
  void reset_batch(int ninst);
  // The standard guess has just been written into b.P (or, with have_std
  // false, a guess without a standard reference was used).
  void begin_step(const Batch& b, bool have_std);
  // Adds the predicted residual to b.P; false when no trained model applies
  // or the prediction was rejected (b.P then holds the standard guess).
  bool predict(const Batch& b);
  // After convergence: residual rows of this step go to the replay buffer.
  void record(const Batch& b);
  // Full-batch Adam steps on the replay buffer; returns the loss before the
  // last step (negative when there is nothing to train on).
  float train(int steps, hipStream_t s);
  bool trained() const { return adam_steps_ > 0; }
  void save(const std::string& path);
  void load(const std::string& path);
  // The same model record inside a larger file: read() checks it into host
  // memory without touching the model, apply() installs it.
  struct Saved {
    int din = 0, dout = 0, bmax = 0;
    std::vector<int> types;
    float scale = 0.f;
    long adam_steps = 0;
    std::vector<float> theta, m, v;
  };
  void save(std::ostream& f);
  static Saved read(std::istream& f);
  void apply(const Saved& r);
  // The run state a resumed run needs to predict and train as the
  // uninterrupted one: the last residual, the previous geometry and the
  // replay buffer (host copies; apply_run after apply, on a batch of mtot).
  struct RunState {
    int have_prev = 0;
    std::vector<double> rprev, xyz_prev;
    int next = 0, count = 0;
    std::vector<int> rows;
    std::vector<double> cnt;
    std::vector<std::vector<float>> X, T, M;
  };
  void save_run(std::ostream& f, long long mtot);
  static RunState read_run(std::istream& f, int din, int dout);
  void apply_run(const RunState& r, long long mtot);

  // Direct use of the network (tests): fixed dimensions, parameter access,
  // evaluation and full-batch training on caller rows (host arrays).
  void configure(int din, int dout, unsigned seed);
  // configure() for a network that belongs to no batch: no element types, no
  // block size and no recorded steps, so the in-run guess sizes a new model
  // from its batch before using one
  void configure_detached(int din, int dout, unsigned seed);
  int din() const { return din_; }
  int dout() const { return dout_; }
  long nparams() const;
  void set_params(const float* h, long n, hipStream_t s);
  void get_params(float* h, long n, hipStream_t s);
  // Y (rows x dout) = net(X); with T and M also the loss and the flat
  // gradient (may be null).
  void eval_rows(int rows, const float* X, const float* T, const float* M, float* Y,
                 float* grad, float* loss, hipStream_t s);
  // steps of Adam (learning rate lr) on caller rows from the current
  // moments; loss before the last step.
  float fit_rows(int rows, const float* X, const float* T, const float* M, int steps, float lr,
                 hipStream_t s);
  // Y = net(X) for device rows X (rows x din) into device Y (rows x dout),
  // enqueued on s with no allocation and no synchronisation; the activations
  // go to the per-GPU array of init_noalloc_scratch (calls that overlap on one
  // GPU race on it).
  void eval_noalloc(int device, int rows, const float* X, float* Y, hipStream_t s);

 private:
  struct Row {
    int inst, a, b, type;   // global atoms a, b
  };
  void ensure_model(const Batch& b);
  void build_rows(const Batch& b);
  void features(const Batch& b, float* X);   // device rows of the current row list
  void forward(int rows, const float* X, hipStream_t s);
  void forward_into(int rows, const float* X, float* h1, float* h2, float* y, hipStream_t s);
  float backward(int rows, const float* X, const float* T, const float* M, double cnt,
                 hipStream_t s);
  void adam(float lr, hipStream_t s);
  void alloc_work(int rows);

  int ninst_ = 0;
  int din_ = 0, dout_ = 0, bmax_ = 0;
  std::vector<int> types_;   // element-pair type table: Z values present
  float scale_ = 0.f;        // residual scale (1 / rms of the first recorded residual)
  long adam_steps_ = 0;
  float lr_ = 1e-3f;
  Buf<float> theta_, grad_, m_, v_;
  // activations of the last forward pass
  Buf<float> h1_, h2_, y_, dy_, dh2_, dh1_;
  Buf<double> lossacc_;
  int work_rows_ = 0;
  // current rows and their device table
  std::vector<Row> rows_;
  std::vector<int> rowinfo_h_;   // per row: 8 ints (see mlp.hip)
  std::vector<float> geo_h_;
  Buf<int> rowinfo_;
  Buf<float> geo_, X_;
  // standard guess and previous residual of every instance (device, mtot)
  Buf<double> pstd_, rprev_, r_;
  bool have_std_ = false, have_prev_ = false;
  std::vector<double> xyz_prev_;
  // replay buffer: features, targets, masks and masked-entry counts per step
  struct Step {
    Buf<float> X, T, M;
    int rows = 0;
    double cnt = 0;
  };
  Step replay_[kReplaySteps];
  int replay_next_ = 0, replay_count_ = 0;
  Buf<float> tx_, tt_, tm_;   // concatenated training rows
};

}  // namespace mlp
}  // namespace bscf
