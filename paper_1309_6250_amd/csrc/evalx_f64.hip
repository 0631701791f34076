// Forward-evaluation kernels of the other representations (Lagrange weights, five separate
// tables, Bloch orbitals) instantiated for f64 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_evalx_f64(int mode, int var, int g, int opl) { return pick_mode_variant<double>(mode, var, g, opl); }

}  // namespace pws
