// Kernels of the steps around the altGDmin loop (Algorithm 1 of the paper:
// the mean image and the residuals; Algorithm 3: the modelling-error
// corrections):
//
//  * the mean image's normal operator: sum_k A_k^H A_k z equals
//    sum_c conj(s_c) o F^H (cnt o F(s_c o z)), cnt(i) the number of frames
//    that sample k-space location i (for full-readout lines F = F_y: the
//    unitary kx transform cancels); k_count_scale applies cnt;
//  * conjugate-gradient bookkeeping in FP64 scalars over FP32 vectors, for
//    one system (the mean) or one system per frame (MEC-1), with every
//    reduction in a fixed order (per-workgroup partials summed by index);
//  * ISTA for MEC-2: the unitary DFT along the frames of every pixel
//    (k_tdft, direct summation from an LDS table, q <= 128), the complex
//    soft threshold, and the threshold / convergence reductions.
#include "kernels_mri.hpp"

namespace ag {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// the mean image's normal operator: scale k-space coil images by the count of
// frames sampling each location.  T is nc images of n values; the location of
// entry p is p / loc_div (loc_div = nx for full-readout lines: one count per
// phase-encode row ky; 1 for general masks).
// ---------------------------------------------------------------------------
__global__ void k_count_scale(float2* T, long n, int nc, int loc_div, const int32_t* loc_ptr, const DevState* st) {
  if (st->err) return;
  const long total = n * nc;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long p = i % n;
    const long loc = p / loc_div;
    const float cnt = (float)(loc_ptr[loc + 1] - loc_ptr[loc]);
    const float2 v = T[i];
    T[i] = make_float2(v.x * cnt, v.y * cnt);
  }
}

// out[p] = sum_k X[k n + p] (frames summed in order, in FP64)
__global__ void k_colsum(const float2* X, long n, int q, float2* out, const DevState* st) {
  if (st->err) return;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < q; ++k) {
      const float2 v = X[(long)k * n + p];
      re += v.x;
      im += v.y;
    }
    out[p] = make_float2((float)re, (float)im);
  }
}

// part[b] = Re <a, b> over this workgroup's slice (a == b: squared norm)
__global__ __launch_bounds__(256) void k_dot_parts(const float2* a, const float2* b, long n, double* part,
                                                   const DevState* st) {
  __shared__ double sh[256];
  if (st->err) return;
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 u = a[i], v = b[i];
    s += (double)u.x * v.x + (double)u.y * v.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ __forceinline__ double sum_parts(const double* part, int nb) {
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  return s;
}

// gamma = ||s_0||^2 after the initial residual's A^H
__global__ void k_cg_start(const double* part, int nb, CgState* cs, const DevState* st) {
  if (threadIdx.x != 0 || st->err) return;
  const double g = sum_parts(part, nb);
  cs->gamma = g;
  cs->gamma0 = g;
  cs->alpha = 0.0;
  cs->beta = 0.0;
  cs->iters = 0;
  cs->done = !(g > 0.0);
}

// alpha = gamma / <p, A^H A p>  (= gamma / ||A p||^2)
__global__ void k_cg_alpha(const double* part, int nb, CgState* cs, const DevState* st) {
  if (threadIdx.x != 0 || st->err || cs->done) return;
  const double d = sum_parts(part, nb);
  if (!(d > 0.0)) {
    cs->done = 1;
    cs->alpha = 0.0;
    return;
  }
  cs->alpha = cs->gamma / d;
}

// x += alpha p; s -= alpha w; part = ||s||^2 over the workgroup's slice
__global__ __launch_bounds__(256) void k_cg_update_xs(float2* x, float2* s, const float2* p, const float2* w, long n,
                                                      const CgState* cs, double* part, const DevState* st) {
  __shared__ double sh[256];
  if (st->err || cs->done) return;
  const float a = (float)cs->alpha;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 pv = p[i], wv = w[i], xv = x[i];
    float2 sv = s[i];
    x[i] = make_float2(xv.x + a * pv.x, xv.y + a * pv.y);
    sv = make_float2(sv.x - a * wv.x, sv.y - a * wv.y);
    s[i] = sv;
    acc += (double)sv.x * sv.x + (double)sv.y * sv.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// gamma' = ||s||^2; one more iteration done; stop when ||s|| <= tol ||s_0||,
// else beta = gamma'/gamma
__global__ void k_cg_beta(const double* part, int nb, double tol, CgState* cs, const DevState* st) {
  if (threadIdx.x != 0 || st->err || cs->done) return;
  const double g = sum_parts(part, nb);
  cs->iters += 1;
  if (sqrt(g) <= tol * sqrt(cs->gamma0)) {
    cs->done = 1;
    return;
  }
  cs->beta = g / cs->gamma;
  cs->gamma = g;
}

// p = s + beta p
__global__ void k_cg_update_p(float2* p, const float2* s, long n, const CgState* cs, const DevState* st) {
  if (st->err || cs->done) return;
  const float b = (float)cs->beta;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 sv = s[i], pv = p[i];
    p[i] = make_float2(sv.x + b * pv.x, sv.y + b * pv.y);
  }
}

// ---------------------------------------------------------------------------
// one CGLS per frame (MEC-1): vectors are n x q (images, column k = frame k)
// or q x len (the padded measurements of frame k); per-frame FP64 scalars.
// Grid (NBF, q): part[k * NBF + b] is workgroup b's share of frame k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_frame_norm_parts(const float2* v, long len, double* part, const DevState* st) {
  __shared__ double sh[256];
  if (st->err) return;
  const int k = blockIdx.y;
  const float2* f = v + (long)k * len;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    const float2 u = f[i];
    acc += (double)u.x * u.x + (double)u.y * u.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)k * gridDim.x + blockIdx.x] = acc;
}

// per frame: gamma = gamma0 = ||s_k||^2 (start), or alpha = gamma / ||A p||^2,
// or gamma' / beta / stop (see the single-system kernels above)
__global__ void k_frames_cg(const double* part, int nb, int q, int mode, double tol, FrameCg* fc, const DevState* st) {
  if (st->err) return;
  for (int k = threadIdx.x; k < q; k += blockDim.x) {
    const double v = sum_parts(part + (long)k * nb, nb);
    FrameCg& c = fc[k];
    if (mode == 0) {
      c.gamma = v;
      c.gamma0 = v;
      c.alpha = 0.0;
      c.beta = 0.0;
      c.done = !(v > 0.0);
      c.iters = 0;
    } else if (mode == 1) {
      if (c.done) continue;
      if (!(v > 0.0)) {
        c.done = 1;
        c.alpha = 0.0;
      } else {
        c.alpha = c.gamma / v;
      }
    } else {
      if (c.done) continue;
      c.iters += 1;
      if (sqrt(v) <= tol * sqrt(c.gamma0)) {
        c.done = 1;
        c.beta = 0.0;
      } else {
        c.beta = v / c.gamma;
        c.gamma = v;
      }
    }
  }
}

// x_k += sign alpha_k p_k (frames in grid.y) for the frames still running:
// launched between the step-length and the stop test of an iteration, so a
// frame that stops at this iteration's test still takes its update
__global__ void k_frames_axpy(float2* x, const float2* p, long len, const FrameCg* fc, int sign, const DevState* st) {
  if (st->err) return;
  const int k = blockIdx.y;
  const FrameCg& c = fc[k];
  if (c.done) return;
  const float a = (float)(sign * c.alpha);
  float2* xf = x + (long)k * len;
  const float2* pf = p + (long)k * len;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    const float2 pv = pf[i], xv = xf[i];
    xf[i] = make_float2(xv.x + a * pv.x, xv.y + a * pv.y);
  }
}

// p_k = s_k + beta_k p_k for the frames still running
__global__ void k_frames_pupdate(float2* p, const float2* s, long len, const FrameCg* fc, const DevState* st) {
  if (st->err) return;
  const int k = blockIdx.y;
  if (fc[k].done) return;
  const float b = (float)fc[k].beta;
  float2* pf = p + (long)k * len;
  const float2* sf = s + (long)k * len;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    const float2 sv = sf[i], pv = pf[i];
    pf[i] = make_float2(sv.x + b * pv.x, sv.y + b * pv.y);
  }
}

// ---------------------------------------------------------------------------
// residuals and small vector operations
// ---------------------------------------------------------------------------
// Z[:, k] = (X[:, k] or 0) + (zbar or 0)
__global__ void k_form_z(const float2* X, const float2* zbar, long n, int q, float2* Z, const DevState* st) {
  if (st->err) return;
  const long total = n * q;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    float2 v = X ? X[i] : make_float2(0.f, 0.f);
    if (zbar) {
      const float2 z = zbar[i % n];
      v = make_float2(v.x + z.x, v.y + z.y);
    }
    Z[i] = v;
  }
}

// out = y - out on every frame's valid samples, 0 on the padding
__global__ void k_sub_from(const float2* y, float2* out, const int32_t* m_k, int nc, int m_max, int q,
                           const DevState* st) {
  if (st->err) return;
  const long total = (long)q * nc * m_max;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m_max);
    const int k = (int)(e / ((long)nc * m_max));
    float2 v = make_float2(0.f, 0.f);
    if (i < m_k[k]) {
      const float2 a = y[e], b = out[e];
      v = make_float2(a.x - b.x, a.y - b.y);
    }
    out[e] = v;
  }
}

// Z[:, k] = (zbar or 0) + U b_k (when U) + (E[:, k] or 0): the output
// assembly of Algorithm 1 (z_k = zbar + x_k + e_k), U n x r column-major,
// B r x q column-major
__global__ void k_expand(const float2* U, const float2* B, const float2* zbar, const float2* E, long n, int q, int r,
                         float2* Z, const DevState* st) {
  if (st->err) return;
  const long total = n * q;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long p = i % n;
    const int k = (int)(i / n);
    float re = 0.f, im = 0.f;
    if (U) {
      for (int j = 0; j < r; ++j) {
        const float2 u = U[(long)j * n + p], b = B[(long)k * r + j];
        re += u.x * b.x - u.y * b.y;
        im += u.x * b.y + u.y * b.x;
      }
    }
    if (zbar) {
      re += zbar[p].x;
      im += zbar[p].y;
    }
    if (E) {
      re += E[i].x;
      im += E[i].y;
    }
    Z[i] = make_float2(re, im);
  }
}

// a += b
__global__ void k_add(float2* a, const float2* b, long n, const DevState* st) {
  if (st->err) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 u = a[i], v = b[i];
    a[i] = make_float2(u.x + v.x, u.y + v.y);
  }
}

__global__ void k_zero2(float2* a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = make_float2(0.f, 0.f);
}

__global__ void k_copy2(const float2* a, float2* b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// ISTA (MEC-2)
// ---------------------------------------------------------------------------
// The unitary DFT along the frames of each pixel: out[k n + p] =
// q^{-1/2} sum_t in[t n + p] exp(-+2 pi i k t / q).  A workgroup stages 64
// pixels x q frames in LDS; thread (pixel, slice) forms every 4th output.
// THRESH: the input is first soft-thresholded by omega (s/|s| (|s| - omega)
// where |s| > omega, else 0), the step of Algorithm 3 before the inverse DFT.
template <bool INV, bool THRESH>
__global__ __launch_bounds__(256) void k_tdft(const float2* in, float2* out, long n, int q, const IstaState* is,
                                              const DevState* st) {
  __shared__ float2 tile[128 * 64];
  __shared__ float2 tw[128];
  if (st->err || is->done) return;
  const int tid = threadIdx.x, pl = tid & 63, sl = tid >> 6;
  const long p0 = (long)blockIdx.x * 64;
  const float om = THRESH ? (float)is->omega : 0.f;
  for (int e = tid; e < q; e += 256) {
    double sv, cv;
    sincospi(2.0 * (double)e / (double)q, &sv, &cv);
    tw[e] = make_float2((float)cv, INV ? (float)sv : -(float)sv);
  }
  for (int e = tid; e < q * 64; e += 256) {
    const int t = e >> 6, pp = e & 63;
    const long p = p0 + pp;
    float2 v = p < n ? in[(long)t * n + p] : make_float2(0.f, 0.f);
    if (THRESH) {
      const float m = sqrtf(v.x * v.x + v.y * v.y);
      const float f = m > om ? (m - om) / m : 0.f;
      v = make_float2(v.x * f, v.y * f);
    }
    tile[t * 64 + pp] = v;
  }
  __syncthreads();
  const long p = p0 + pl;
  if (p >= n) return;
  const float sc = rsqrtf((float)q);
  for (int k = sl; k < q; k += 4) {
    float re = 0.f, im = 0.f;
    int m = 0;  // (k t) mod q
    for (int t = 0; t < q; ++t) {
      const float2 v = tile[t * 64 + pl], w = tw[m];
      re += v.x * w.x - v.y * w.y;
      im += v.x * w.y + v.y * w.x;
      m += k;
      if (m >= q) m -= q;
    }
    out[(long)k * n + p] = make_float2(re * sc, im * sc);
  }
}

// part[b] = max |v| over the workgroup's slice
__global__ __launch_bounds__(256) void k_absmax_parts(const float2* v, long len, double* part, const IstaState* is,
                                                      const DevState* st) {
  __shared__ double sh[256];
  if (st->err || is->done) return;
  double m = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    const float2 u = v[i];
    m = fmax(m, sqrt((double)u.x * u.x + (double)u.y * u.y));
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// part[2b] = ||a - b||^2, part[2b+1] = ||b||^2 over the workgroup's slice
__global__ __launch_bounds__(256) void k_change_parts(const float2* a, const float2* b, long len, double* part,
                                                      const IstaState* is, const DevState* st) {
  __shared__ double sh[256];
  if (st->err || is->done) return;
  double d = 0.0, r = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    const float2 u = a[i], v = b[i];
    const double dx = (double)u.x - v.x, dy = (double)u.y - v.y;
    d += dx * dx + dy * dy;
    r += (double)v.x * v.x + (double)v.y * v.y;
  }
  d = block_sum(d, sh);
  r = block_sum(r, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = d;
    part[2 * blockIdx.x + 1] = r;
  }
}

// t = 0: omega = frac * max |M_0|.  t >= 1: stop after this update when
// ||M_t - M_{t-1}|| / ||M_{t-1}|| < tol.
__global__ void k_ista_step(const double* part, int nb, int t, double frac, double tol, IstaState* is,
                            const DevState* st) {
  if (threadIdx.x != 0 || st->err || is->done) return;
  if (t == 0) {
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, part[b]);
    is->omega = frac * m;
    is->stop_next = 0;
  } else {
    double d = 0.0, r = 0.0;
    for (int b = 0; b < nb; ++b) {
      d += part[2 * b];
      r += part[2 * b + 1];
    }
    const double ch = r > 0.0 ? sqrt(d / r) : 0.0;
    is->last_change = ch;
    is->stop_next = ch < tol;
  }
}

// after the update of iteration t: count it, and stop if the test said so
__global__ void k_ista_commit(IstaState* is, const DevState* st) {
  if (threadIdx.x != 0 || st->err || is->done) return;
  is->iters += 1;
  if (is->stop_next) is->done = 1;
}

__global__ void k_ista_reset(IstaState* is) {
  if (threadIdx.x != 0) return;
  is->omega = 0.0;
  is->last_change = 0.0;
  is->iters = 0;
  is->done = 0;
  is->stop_next = 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tdft(const float2* in, float2* out, long n, int q, bool inv, bool thresh, const IstaState* is,
                       const DevState* st, hipStream_t s) {
  const dim3 g((unsigned)((n + 63) / 64));
  if (!inv && !thresh) hipLaunchKernelGGL((k_tdft<false, false>), g, dim3(256), 0, s, in, out, n, q, is, st);
  else if (inv && thresh) hipLaunchKernelGGL((k_tdft<true, true>), g, dim3(256), 0, s, in, out, n, q, is, st);
  else if (inv) hipLaunchKernelGGL((k_tdft<true, false>), g, dim3(256), 0, s, in, out, n, q, is, st);
  else hipLaunchKernelGGL((k_tdft<false, true>), g, dim3(256), 0, s, in, out, n, q, is, st);
  return hipGetLastError();
}

}  // namespace ag
