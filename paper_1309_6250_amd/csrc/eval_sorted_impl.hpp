// Locality-ordered forward evaluation (spline_eval_vgl_sorted).
//
// Points arrive in any order (walkers x electrons, spread over the whole cell), so consecutive
// points rarely share table rows and every block is gathered from memory.  On average a row of the
// table belongs to the blocks of several points (64 P / N1 N2 N3 of them), so evaluating the points
// in the order of a space-filling curve over the grid cells lets the points that one workgroup,
// and one XCD, handle in sequence find most rows of their blocks already in L2 or the Infinity
// Cache.  Steps: a Morton key of each point's cell (three 10-bit indices interleaved), a stable
// radix sort of (key, point index), then the forward kernel through the resulting permutation.
// Workgroups are dispatched to the 8 XCDs in turn, so workgroup b takes tile (b mod 8) * per_xcd +
// b / 8: each XCD walks a contiguous stretch of the curve.  Each point's outputs go to its own
// row, in the caller's order; the arithmetic is that of k_eval, so results are bitwise identical.
#pragma once
#include "eval_impl.hpp"

namespace pws {

template <typename TS, int MODE, int G, int OPL>
__global__ __launch_bounds__(256) void k_eval_perm(EvalArgs a, const int32_t* perm, int32_t per_xcd) {
  constexpr int GPB = 256 / G;
  const int b = (int)blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  const int64_t q = (int64_t)tile * GPB + (int)threadIdx.x / G;
  if (q >= a.n_pts) return;
  int p = perm[q];
  if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
  eval_point<TS, MODE, G, OPL, 0>(a, p, (int)threadIdx.x % G);
}

typedef void (*PermKernel)(EvalArgs, const int32_t*, int32_t);

template <typename TS, int MODE, int OPL>
inline PermKernel pick_perm_g(int g) {
  switch (g) {
    case 2: return k_eval_perm<TS, MODE, 2, OPL>;
    case 4: return k_eval_perm<TS, MODE, 4, OPL>;
    case 8: return k_eval_perm<TS, MODE, 8, OPL>;
    case 16: return k_eval_perm<TS, MODE, 16, OPL>;
    case 32: return k_eval_perm<TS, MODE, 32, OPL>;
    case 64: return k_eval_perm<TS, MODE, 64, OPL>;
    case 128: return k_eval_perm<TS, MODE, 128, OPL>;
    case 256: return k_eval_perm<TS, MODE, 256, OPL>;
    default: return nullptr;
  }
}

template <typename TS, int MODE>
inline PermKernel pick_perm_opl(int g, int opl) {
  if (opl == OplSet<TS>::lo) return pick_perm_g<TS, MODE, OplSet<TS>::lo>(g);
  if (opl == OplSet<TS>::mid) return pick_perm_g<TS, MODE, OplSet<TS>::mid>(g);
  if (opl == OplSet<TS>::hi) return pick_perm_g<TS, MODE, OplSet<TS>::hi>(g);
  return nullptr;
}

template <typename TS>
inline PermKernel pick_perm_mode(int mode, int g, int opl) {
  switch (mode) {
    case MODE_V: return pick_perm_opl<TS, MODE_V>(g, opl);
    case MODE_VGL: return pick_perm_opl<TS, MODE_VGL>(g, opl);
    case MODE_VGL_SEPLAP: return pick_perm_opl<TS, MODE_VGL_SEPLAP>(g, opl);
    default: return nullptr;
  }
}

}  // namespace pws
