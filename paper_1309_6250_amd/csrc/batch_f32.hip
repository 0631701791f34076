// Batched persistent VGL kernels instantiated for f32 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

BatchKernel pick_batch_f32(int mode, int g, int opl) { return pick_batch_mode<float>(mode, g, opl); }

}  // namespace pws
