// Locality-ordered forward-evaluation kernels instantiated for f64 coefficient tables.
#include "eval_sorted_impl.hpp"

namespace pws {

PermKernel pick_perm_f64(int mode, int g, int opl) { return pick_perm_mode<double>(mode, g, opl); }

}  // namespace pws
