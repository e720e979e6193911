// Kernel instantiations for the d2q9_paper lattice and basis, f64 storage.
#include "launch.hpp"

namespace lbmrv {
LBMRV_DEFINE_LAUNCHERS(d2q9_paper, BasisD2Q9Paper, f64, 0)
}  // namespace lbmrv
