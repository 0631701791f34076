// Forward-evaluation kernels instantiated for f64 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_eval_f64(int mode, int g, int opl) { return pick_mode<double>(mode, g, opl); }

}  // namespace pws
