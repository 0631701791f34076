// Batched persistent VGL kernels instantiated for bf16 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

BatchKernel pick_batch_bf16(int mode, int g, int opl) { return pick_batch_mode<uint16_t>(mode, g, opl); }

}  // namespace pws
