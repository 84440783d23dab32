// Kernels and launches of the 7-point stencil with Hermite order 3.
#include "launch_impl.hpp"

namespace lbsmrt {
template struct Launch<7, 3>;
}  // namespace lbsmrt
