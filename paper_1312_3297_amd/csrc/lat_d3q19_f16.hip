// Kernel instantiations for the d3q19 lattice and basis, f16 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d3q19, BasisD3Q19, f16, 2)
}  // namespace lbmrv
