// Kernel instantiations for the d3q19 lattice and basis, f64 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d3q19, BasisD3Q19, f64, 0)
}  // namespace lbmrv
