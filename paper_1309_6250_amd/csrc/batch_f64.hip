// Batched persistent VGL kernels instantiated for f64 coefficient tables.
#include "eval_impl.hpp"

namespace pws {

BatchKernel pick_batch_f64(int mode, int g, int opl) { return pick_batch_mode<double>(mode, g, opl); }

}  // namespace pws
