// Declarations shared by the cell-wise work (cells.hip) and the C ABI (abi.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pwspline.h"

namespace pws {

// Targets and weights of spline_fit_terms_cells: values and Laplacians (NULL target: no term).
struct FitTerms {
  const void* t_v;
  double w_v;
  const void* t_lap;
  double w_lap;
  double* loss;
};

int cells_eval_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);
// fit == NULL: plain outputs; else v and lap receive the misfit's upstream gradients
int launch_eval_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                      void* lap, void* work, int64_t work_bytes, bool reuse, hipStream_t stream,
                      const FitTerms* fit);
int fit_gradient_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);
// the fit's data terms and their coefficient gradient in one pass (FP32 tables, dense points)
int launch_fit_gradient(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* t_v,
                        double w_v, const void* t_lap, double w_lap, void* gtable, double* loss, void* work,
                        int64_t work_bytes, bool reuse, hipStream_t stream);

}  // namespace pws
