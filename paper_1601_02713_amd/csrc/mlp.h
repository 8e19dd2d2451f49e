// Learned SCF guess: per-atom-pair MLP predicting density blocks (mlp.hip).
#pragma once
#include <string>
#include <vector>

struct bscf_ctx;

namespace bscf {
namespace mlp {

class Guess {
 public:
  void reset_batch(int ninst);
  // writes a predicted density into the context's P; false if unavailable
  bool predict(bscf_ctx* c);
  // records the converged densities of the last SCF as training data
  void record(bscf_ctx* c);
  float train(bscf_ctx* c, int steps);
  void save(const std::string& path);
  void load(const std::string& path);

 private:
  int ninst_ = 0;
  bool trained_ = false;
};

}  // namespace mlp
}  // namespace bscf
