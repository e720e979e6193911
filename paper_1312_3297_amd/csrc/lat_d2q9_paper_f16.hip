// Kernel instantiations for the d2q9_paper lattice and basis, f16 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d2q9_paper, BasisD2Q9Paper, f16, 2)
}  // namespace lbmrv
