// Kernel instantiations for the d2q9_geier lattice and basis, f32 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d2q9_geier, BasisD2Q9Geier, f32, 1)
}  // namespace lbmrv
