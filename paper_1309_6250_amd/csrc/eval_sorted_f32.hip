// Locality-ordered forward-evaluation kernels instantiated for f32 coefficient tables.
#include "eval_sorted_impl.hpp"

namespace pws {

PermKernel pick_perm_f32(int mode, int g, int opl) { return pick_perm_mode<float>(mode, g, opl); }

}  // namespace pws
