// Forward-evaluation kernels instantiated for f32 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_eval_f32(int mode, int g, int opl) { return pick_mode<float>(mode, g, opl); }

}  // namespace pws
