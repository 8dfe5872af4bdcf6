// FP32 / complex64 instantiation of every kernel.
#include "launch_impl.hpp"

namespace ctfiss {
CTFISS_INSTANTIATE(float)
}  // namespace ctfiss
