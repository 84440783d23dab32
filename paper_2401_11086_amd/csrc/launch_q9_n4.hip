// Kernels and launches of the 9-point stencil with Hermite order 4.
#include "launch_impl.hpp"

namespace lbsmrt {
template struct Launch<9, 4>;
}  // namespace lbsmrt
