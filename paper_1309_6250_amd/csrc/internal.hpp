// Internal declarations shared by the library's translation units (not part of the C ABI).
#pragma once
#include "eval_impl.hpp"

namespace pws {

int vec_of(int dtype);
void opl_set(int dtype, int out[3]);
bool tile_valid(int dtype, const int32_t tile[2]);
bool tile_valid_for(const spl_desc* d, const int32_t tile[2]);
void default_tile(const spl_desc* d, int32_t tile[2]);
void tile_for(const spl_desc* d, int32_t tile[2]);
int check_eval_args(const spl_desc* d, const void* table, int64_t n_pts, const double* pos);
int check_vgl_outputs(const spl_desc* d, const void* v, const void* grad, const void* lap);
void fill_eval_args(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                    void* lap, int values_only, int opl, EvalArgs* a);
int launch_eval(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                void* lap, int values_only, const int32_t tile[2], hipStream_t stream);

int sorted_eval_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);
int launch_eval_sorted(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                       void* lap, int values_only, const int32_t tile[2], void* work, int64_t work_bytes,
                       hipStream_t stream);

BatchKernel pick_batch_f64(int mode, int g, int opl);
BatchKernel pick_batch_f32(int mode, int g, int opl);
BatchKernel pick_batch_bf16(int mode, int g, int opl);

}  // namespace pws
