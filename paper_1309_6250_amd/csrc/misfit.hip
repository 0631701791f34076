// spline_misfit: the data term of the least-squares fit of coefficients to orbital samples.
//
// For n outputs y (values or Laplacians of the spline at the fit points) and their targets t:
//     loss += w sum_i (y_i - t_i)^2,        g_i = 2 w (y_i - t_i),
// g being the upstream gradient that spline_eval_vgl_backward turns into the gradient of the
// loss with respect to the coefficients.  One pass over y and t, HBM-bound.
//
// The sum is formed in FP64 and in a fixed order: MISFIT_BLOCKS workgroups each own the same
// grid-strided elements on every call and reduce them in a fixed tree in LDS; one workgroup
// then adds the partial sums in a fixed tree and the result to *loss.  So the loss is
// reproducible bit for bit, like the deterministic adjoint it feeds.
#include <cmath>

#include "common.hpp"

namespace pws {

constexpr int MISFIT_BLOCKS = 1024;
constexpr int MISFIT_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(MISFIT_THREADS) void k_misfit(int64_t n, const T* y, const T* t, T two_w, T* g,
                                                           double* partial) {
  __shared__ double red[MISFIT_THREADS];
  const int64_t stride = (int64_t)MISFIT_BLOCKS * MISFIT_THREADS;
  double s = 0.0;
  int64_t i = (int64_t)blockIdx.x * MISFIT_THREADS + threadIdx.x;
  // four independent loads in flight per thread
  for (; i + 3 * stride < n; i += 4 * stride) {
    T r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = y[i + u * stride] - t[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s += (double)r[u] * (double)r[u];
      g[i + u * stride] = two_w * r[u];
    }
  }
  for (; i < n; i += stride) {
    const T r = y[i] - t[i];
    s += (double)r * (double)r;
    g[i] = two_w * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = MISFIT_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(MISFIT_THREADS) void k_misfit_total(const double* partial, double w, double* loss) {
  __shared__ double red[MISFIT_THREADS];
  double s = 0.0;
  for (int b = threadIdx.x; b < MISFIT_BLOCKS; b += MISFIT_THREADS) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = MISFIT_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss += w * red[0];
}

}  // namespace pws

using namespace pws;

extern "C" {

int spline_misfit_work_bytes(const spl_desc* d, int64_t n, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (n < 0 || !bytes) return fail(SPL_EINVAL, "n < 0 or bytes is NULL");
  *bytes = (int64_t)MISFIT_BLOCKS * (int64_t)sizeof(double);
  return SPL_OK;
}

int spline_misfit(const spl_desc* d, int64_t n, const void* y, const void* t, double w, void* g, double* loss,
                  void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (n < 0) return fail(SPL_EINVAL, "n < 0");
  if (!std::isfinite(w)) return fail(SPL_EINVAL, "weight is not finite");
  if (n == 0) return SPL_OK;
  if (!y || !t || !g || !loss || !work) return fail(SPL_EINVAL, "NULL y, t, g, loss or work");
  if (work_bytes < (int64_t)MISFIT_BLOCKS * (int64_t)sizeof(double))
    return fail(SPL_EINVAL, "work must hold %d bytes", MISFIT_BLOCKS * (int)sizeof(double));
  const size_t es = d->dtype == SPL_F64 ? 8 : 4;
  for (const void* p : {y, t, static_cast<const void*>(g)})
    if ((uintptr_t)p % es) return fail(SPL_EINVAL, "y, t and g must be aligned to their element size");
  if ((uintptr_t)loss % 8 || (uintptr_t)work % 8) return fail(SPL_EINVAL, "loss and work must be 8-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(work);
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_misfit<double>, dim3(MISFIT_BLOCKS), dim3(MISFIT_THREADS), 0, s, n,
                       static_cast<const double*>(y), static_cast<const double*>(t), 2.0 * w,
                       static_cast<double*>(g), partial);
  else
    hipLaunchKernelGGL(k_misfit<float>, dim3(MISFIT_BLOCKS), dim3(MISFIT_THREADS), 0, s, n,
                       static_cast<const float*>(y), static_cast<const float*>(t), (float)(2.0 * w),
                       static_cast<float*>(g), partial);
  if ((rc = hip_fail(hipGetLastError(), "misfit launch"))) return rc;
  hipLaunchKernelGGL(k_misfit_total, dim3(1), dim3(MISFIT_THREADS), 0, s, partial, w, loss);
  return hip_fail(hipGetLastError(), "misfit total launch");
}

}  // extern "C"
