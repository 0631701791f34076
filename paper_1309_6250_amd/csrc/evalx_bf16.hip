// Forward-evaluation kernels of the other representations (Lagrange weights, five separate
// tables, Bloch orbitals) instantiated for bf16 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_evalx_bf16(int mode, int var, int g, int opl) { return pick_mode_variant<uint16_t>(mode, var, g, opl); }

}  // namespace pws
