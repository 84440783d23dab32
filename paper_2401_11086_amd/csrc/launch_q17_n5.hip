// Kernels and launches of the 17-point stencil with Hermite order 5.
#include "launch_impl.hpp"

namespace lbsmrt {
template struct Launch<17, 5>;
}  // namespace lbsmrt
