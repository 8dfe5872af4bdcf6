// FP64 / complex128 instantiation of every kernel.
#include "launch_impl.hpp"

namespace ctfiss {
CTFISS_INSTANTIATE(double)
}  // namespace ctfiss
