// Forward-evaluation kernels of the other representations (Lagrange weights, five separate
// tables, Bloch orbitals) instantiated for f32 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_evalx_f32(int mode, int var, int g, int opl) { return pick_mode_variant<float>(mode, var, g, opl); }

}  // namespace pws
