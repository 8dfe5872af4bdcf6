// Mixed precision: FP32 / complex64 ISS kernels whose sweep updates the rows of
// W in FP64 registers.  Every other kernel of the mixed path is the FP32 one.
#include "launch_impl.hpp"

namespace ctfiss {
CTFISS_INSTANTIATE_W(float, true)
}  // namespace ctfiss
