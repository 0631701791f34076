// Forward-evaluation kernels instantiated for bf16 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_eval_bf16(int mode, int g, int opl) { return pick_mode<uint16_t>(mode, g, opl); }

}  // namespace pws
