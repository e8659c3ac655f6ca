// Kernels for one population storage format (see lbpc_device.hpp).
#include "lbpc_launch.hpp"

namespace lbpc {
LBPC_INSTANTIATE(1)
}  // namespace lbpc
