// Device state and kernels of the steps around the altGDmin loop (the mean
// image, residuals, modelling-error corrections); see kernels_mri.hip.
#pragma once

#include "kernels_core.hpp"

namespace ag {

// conjugate gradients on one system (the mean image)
struct CgState {
  double gamma, gamma0, alpha, beta;
  int32_t iters, done;
};

// conjugate gradients on one system per frame (MEC-1)
struct FrameCg {
  double gamma, gamma0, alpha, beta;
  int32_t iters, done;
};

// ISTA (MEC-2)
struct IstaState {
  double omega, last_change;
  int32_t iters, done, stop_next, pad;
};

constexpr int MRI_NB = 256;   // workgroups (and partial sums) of a single-system reduction
constexpr int MRI_NBF = 64;   // workgroups per frame of a per-frame reduction

__global__ void k_count_scale(float2* T, long n, int nc, int loc_div, const int32_t* loc_ptr, const DevState* st);
__global__ void k_colsum(const float2* X, long n, int q, float2* out, const DevState* st);
__global__ void k_dot_parts(const float2* a, const float2* b, long n, double* part, const DevState* st);
__global__ void k_cg_start(const double* part, int nb, CgState* cs, const DevState* st);
__global__ void k_cg_alpha(const double* part, int nb, CgState* cs, const DevState* st);
__global__ void k_cg_update_xs(float2* x, float2* s, const float2* p, const float2* w, long n, const CgState* cs,
                               double* part, const DevState* st);
__global__ void k_cg_beta(const double* part, int nb, double tol, CgState* cs, const DevState* st);
__global__ void k_cg_update_p(float2* p, const float2* s, long n, const CgState* cs, const DevState* st);
__global__ void k_frame_norm_parts(const float2* v, long len, double* part, const DevState* st);
__global__ void k_frames_cg(const double* part, int nb, int q, int mode, double tol, FrameCg* fc, const DevState* st);
__global__ void k_frames_axpy(float2* x, const float2* p, long len, const FrameCg* fc, int sign, const DevState* st);
__global__ void k_frames_pupdate(float2* p, const float2* s, long len, const FrameCg* fc, const DevState* st);
__global__ void k_form_z(const float2* X, const float2* zbar, long n, int q, float2* Z, const DevState* st);
__global__ void k_sub_from(const float2* y, float2* out, const int32_t* m_k, int nc, int m_max, int q,
                           const DevState* st);
__global__ void k_add(float2* a, const float2* b, long n, const DevState* st);
__global__ void k_expand(const float2* U, const float2* B, const float2* zbar, const float2* E, long n, int q, int r,
                         float2* Z, const DevState* st);
__global__ void k_zero2(float2* a, long n);
__global__ void k_copy2(const float2* a, float2* b, long n);
__global__ void k_absmax_parts(const float2* v, long len, double* part, const IstaState* is, const DevState* st);
__global__ void k_change_parts(const float2* a, const float2* b, long len, double* part, const IstaState* is,
                               const DevState* st);
__global__ void k_ista_step(const double* part, int nb, int t, double frac, double tol, IstaState* is,
                            const DevState* st);
__global__ void k_ista_commit(IstaState* is, const DevState* st);
__global__ void k_ista_reset(IstaState* is);
hipError_t launch_tdft(const float2* in, float2* out, long n, int q, bool inv, bool thresh, const IstaState* is,
                       const DevState* st, hipStream_t s);

}  // namespace ag
