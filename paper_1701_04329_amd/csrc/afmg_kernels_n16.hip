// The level, coarse and adjoint kernels for boxes of 16^D cells (paper §2.1:
// the box size N is a parameter of the grid), compiled apart from those for
// 8^D cells so that the two builds run in parallel.
#define AFMG_INSTANTIATE_ONLY
#include "afmg_kernels.hip"

namespace afmg {
AFMG_BOX_INST(2, 16)
AFMG_BOX_INST(3, 16)
}  // namespace afmg
