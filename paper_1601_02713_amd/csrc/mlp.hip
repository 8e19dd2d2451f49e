// Learned SCF guess (placeholder until the network is in place).
#include <stdexcept>

#include "mlp.h"

namespace bscf {
namespace mlp {

void Guess::reset_batch(int ninst) { ninst_ = ninst; trained_ = false; }
bool Guess::predict(bscf_ctx*) { return false; }
void Guess::record(bscf_ctx*) {}
float Guess::train(bscf_ctx*, int) { throw std::runtime_error("learned guess not available"); }
void Guess::save(const std::string&) { throw std::runtime_error("learned guess not available"); }
void Guess::load(const std::string&) { throw std::runtime_error("learned guess not available"); }

}  // namespace mlp
}  // namespace bscf
