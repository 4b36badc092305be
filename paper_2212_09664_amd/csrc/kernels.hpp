// Kernel argument blocks and launch helpers shared by the host code and the
// kernel translation units.
#pragma once

#include "common.hpp"

namespace ag {

struct RowArgs {
  const float2* src;
  float2* dst;
  const float2* tw;
  long nrows;
  const int32_t* m_k;  // null: every row valid
  int nc, lmax;        // measurement-line layout when m_k != null
  float scale;
  int trunc;           // zero samples with |v|^2 > gamma before the transform
  int check_halt;
  const DevState* st;
  int32_t* trunc_count;  // non-null with trunc: receives the number of samples zeroed
};

__device__ __forceinline__ bool row_valid(const RowArgs& a, long rho, int N) {
  if (!a.m_k) return true;
  const long per_k = (long)a.nc * a.lmax;
  const int k = (int)(rho / per_k);
  const int l = (int)(rho % a.lmax);
  return l < a.m_k[k] / N;
}

struct ColFwdArgs {
  const float2* src;
  long src_img_stride;
  const float2* coils;
  long n;
  int nx;
  const float2* tw;
  float2* dst;
  long dst_c_stride, dst_img_stride;
  const int32_t* rows;     // ky of each output row
  long rows_img_stride;
  const int32_t* m_k;      // non-null: n_rows = m_k[img]/nx, rows per image
  const int32_t* n_rows_ptr;  // non-null: n_rows = *n_rows_ptr
  int zero_pad_rows;       // > 0: write zeros for rows n_rows..zero_pad_rows-1
  float scale;
  int check_halt;
  const DevState* st;
};

struct ColAdjArgs {
  const float2* src;
  long src_c_stride, src_img_stride;
  const int32_t* rows;
  long rows_img_stride;
  const int32_t* m_k_rows;    // non-null: n_rows = m_k_rows[img]/nx, rows per image
  const int32_t* n_rows_ptr;  // non-null: n_rows = *n_rows_ptr
  const float2* coils;
  long n;
  int nx, nc;
  const float2* tw;
  float2* dst;
  long dst_img_stride;
  int cgs;                    // coils per workgroup (0: all); group g writes dst + g*dst_part_stride
  long dst_part_stride;
  const int32_t* m_k_scale;   // non-null: scale by 1/sqrt(m_k[img] * mbar)
  float scale;
  int accumulate;
  int check_halt;
  const DevState* st;
};

hipError_t launch_rows(int N, const RowArgs& a, bool inv, hipStream_t st);
hipError_t launch_cols(int N, const ColFwdArgs* f, const ColAdjArgs* d, int nx, int n_img, int nc,
                       hipStream_t st);
int col_tile(int N, int nx);
int col_tile_adj(int N, int nx);

__global__ void k_twiddle(float2* tw, int N);
__global__ void k_gather(const float2* img, long img_stride_c, long img_stride_k, const int32_t* mask,
                         const int32_t* m_k, int m_max, int nc, int k0, float2* y, const DevState* st);
__global__ void k_scatter(const float2* y, const int32_t* mask, const int32_t* m_k, int m_max, int nc,
                          int k0, float2* img, long img_stride_c, long img_stride_k, const DevState* st,
                          int trunc, int32_t* trunc_count);
__global__ void k_zero(float2* p, long n);

}  // namespace ag
