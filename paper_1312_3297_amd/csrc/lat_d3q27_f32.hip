// Kernel instantiations for the d3q27 lattice and basis, f32 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d3q27, BasisD3Q27, f32, 1)
}  // namespace lbmrv
