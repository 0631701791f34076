// Locality-ordered forward-evaluation kernels instantiated for bf16 coefficient tables.
#include "eval_sorted_impl.hpp"

namespace pws {

PermKernel pick_perm_bf16(int mode, int g, int opl) { return pick_perm_mode<uint16_t>(mode, g, opl); }

}  // namespace pws
