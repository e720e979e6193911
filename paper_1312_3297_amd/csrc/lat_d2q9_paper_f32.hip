// Kernel instantiations for the d2q9_paper lattice and basis, f32 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d2q9_paper, BasisD2Q9Paper, f32, 1)
}  // namespace lbmrv
