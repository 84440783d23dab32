// Kernels and launches of the 9-point stencil with Hermite order 5.
#include "launch_impl.hpp"

namespace lbsmrt {
template struct Launch<9, 5>;
}  // namespace lbsmrt
