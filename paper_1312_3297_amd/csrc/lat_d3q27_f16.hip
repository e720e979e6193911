// Kernel instantiations for the d3q27 lattice and basis, f16 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d3q27, BasisD3Q27, f16, 2)
}  // namespace lbmrv
