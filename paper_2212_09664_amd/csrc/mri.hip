// Host side of the steps around the altGDmin loop (include/altgdmin.h):
// the mean image and the residual measurements of Algorithm 1, the automatic
// rank of Algorithm 2's parameter setting, and the modelling-error
// corrections of Algorithm 3 (MEC-1 by per-frame CGLS, MEC-2 by ISTA on the
// temporal DFT).  Every step is a launch sequence on the context's stream
// over a caller-provided auxiliary workspace.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ctx.hpp"
#include "kernels_mri.hpp"

using ag_host::map_hip;

// The scratch of altgdmin_mean_noalloc (the CG vectors, the normal operator's
// coil images, the reduction partials and the CG scalars): one copy per GPU,
// held until the process ends.  Host code uses only the device address that
// hipGetSymbolAddress returns for the current device, never this name.
constexpr size_t kMeanScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kMeanScratchBytes];

namespace {

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// the auxiliary workspace, carved from its base
struct Aux {
  float2 *v0, *v1, *v2;  // n x q each
  float2 *y0, *y1;       // q x nc x m_max each
  float2* ci;            // nc x n: coil images of the normal operator
  double* part;          // reduction partials
  CgState* cg;
  FrameCg* fc;           // q
  IstaState* is;
  double* lam;           // 16
};

size_t aux_layout(const altgdmin_ctx* c, char* base, Aux* a) {
  const altgdmin_params& p = c->p;
  const size_t nq = sizeof(float2) * (size_t)c->n * p.q;
  const size_t ys = sizeof(float2) * (size_t)p.q * p.nc * p.m_max;
  const size_t nparts = std::max<size_t>(2 * MRI_NB, (size_t)p.q * MRI_NBF);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = al256(off + b);
    return base ? base + o : nullptr;
  };
  Aux t{};
  t.v0 = reinterpret_cast<float2*>(take(nq));
  t.v1 = reinterpret_cast<float2*>(take(nq));
  t.v2 = reinterpret_cast<float2*>(take(nq));
  t.y0 = reinterpret_cast<float2*>(take(ys));
  t.y1 = reinterpret_cast<float2*>(take(ys));
  t.ci = reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)p.nc * c->n));
  t.part = reinterpret_cast<double*>(take(sizeof(double) * nparts));
  t.cg = reinterpret_cast<CgState*>(take(sizeof(CgState)));
  t.fc = reinterpret_cast<FrameCg*>(take(sizeof(FrameCg) * p.q));
  t.is = reinterpret_cast<IstaState*>(take(sizeof(IstaState)));
  t.lam = reinterpret_cast<double*>(take(sizeof(double) * 16));
  if (a) *a = t;
  return off;
}

bool aux_ok(const void* d_aux) { return d_aux && (reinterpret_cast<uintptr_t>(d_aux) & 255) == 0; }

unsigned grid_for(long n) { return (unsigned)std::max(1L, std::min(1024L, (n + 255) / 256)); }

// out = sum_k A_k^H A_k z = sum_c conj(s_c) o F^H (cnt o F(s_c o z)), with F the
// y transform only for full-readout lines (the kx transform is unitary and
// the mask does not depend on kx)
hipError_t normal_op(altgdmin_ctx* c, const float2* z, float2* out, float2* ci) {
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  ColFwdArgs f{};
  f.src = z;
  f.src_img_stride = c->n;
  f.coils = c->coils;
  f.n = c->n;
  f.nx = p.nx;
  f.tw = c->at<float2>(c->o_twy);
  f.dst = ci;
  f.dst_c_stride = c->n;
  f.dst_img_stride = 0;
  f.scale = (float)(1.0 / sqrt((double)p.ny));
  f.st = c->st();
  hipError_t e = launch_cols(p.ny, &f, nullptr, p.nx, 1, p.nc, s);
  if (e != hipSuccess) return e;
  RowArgs ra{};
  ra.src = ra.dst = ci;
  ra.tw = c->at<float2>(c->o_twx);
  ra.nrows = (long)p.nc * p.ny;
  ra.scale = (float)(1.0 / sqrt((double)p.nx));
  ra.st = c->st();
  if (!c->lines) {
    e = launch_rows(p.nx, ra, false, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_count_scale, dim3(1024), dim3(256), 0, s, ci, (long)c->n, p.nc, c->lines ? p.nx : 1,
                     c->at<int32_t>(c->o_locptr), c->st());
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!c->lines) {
    e = launch_rows(p.nx, ra, true, s);
    if (e != hipSuccess) return e;
  }
  ColAdjArgs d{};
  d.src = ci;
  d.src_c_stride = c->n;
  d.src_img_stride = 0;
  d.coils = c->coils;
  d.n = c->n;
  d.nx = p.nx;
  d.nc = p.nc;
  d.tw = c->at<float2>(c->o_twy);
  d.dst = out;
  d.dst_img_stride = c->n;
  d.scale = (float)(1.0 / sqrt((double)p.ny));
  d.st = c->st();
  return launch_cols(p.ny, nullptr, &d, p.nx, 1, p.nc, s);
}

hipError_t frame_norms(altgdmin_ctx* c, const float2* v, long len, double* part) {
  hipLaunchKernelGGL(k_frame_norm_parts, dim3(MRI_NBF, c->p.q), dim3(256), 0, c->stream, v, len, part, c->st());
  return hipGetLastError();
}

#define AGCHK(x)                     \
  do {                               \
    hipError_t _e = (x);             \
    if (_e != hipSuccess) return _e; \
  } while (0)

hipError_t mean_seq(altgdmin_ctx* c, double tol, int maxit, float2* x, const Aux& a) {
  hipStream_t s = c->stream;
  const long n = c->n;
  float2 *sv = a.v0, *pv = a.v1, *wv = a.v2;
  DevState* st = c->st();
  // s_0 = A^H y = sum_k A_k^H y_k (x_0 = 0)
  float2* T = c->at<float2>(c->o_T);
  AGCHK(ag_host::adjoint_op(c, c->y, T, 0, 0));
  hipLaunchKernelGGL(k_colsum, dim3(grid_for(n)), dim3(256), 0, s, T, n, c->p.q, sv, st);
  hipLaunchKernelGGL(k_zero2, dim3(grid_for(n)), dim3(256), 0, s, x, n);
  hipLaunchKernelGGL(k_copy2, dim3(grid_for(n)), dim3(256), 0, s, sv, pv, n);
  hipLaunchKernelGGL(k_dot_parts, dim3(MRI_NB), dim3(256), 0, s, sv, sv, n, a.part, st);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(1), 0, s, a.part, MRI_NB, a.cg, st);
  AGCHK(hipGetLastError());
  for (int it = 0; it < maxit; ++it) {
    AGCHK(normal_op(c, pv, wv, a.ci));
    hipLaunchKernelGGL(k_dot_parts, dim3(MRI_NB), dim3(256), 0, s, pv, wv, n, a.part, st);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1), 0, s, a.part, MRI_NB, a.cg, st);
    hipLaunchKernelGGL(k_cg_update_xs, dim3(MRI_NB), dim3(256), 0, s, x, sv, pv, wv, n, a.cg, a.part, st);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1), 0, s, a.part, MRI_NB, tol, a.cg, st);
    hipLaunchKernelGGL(k_cg_update_p, dim3(grid_for(n)), dim3(256), 0, s, pv, sv, n, a.cg, st);
    AGCHK(hipGetLastError());
  }
  return hipSuccess;
}

// ---- the no-allocation variant of the mean image ---------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the scratch's device address on the current device (looked up once per device)
altgdmin_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ALTGDMIN_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ALTGDMIN_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ALTGDMIN_OK;
}

// the mean image's buffers carved from a base: three n-vectors, the coil
// images, the partials and the scalars; returns the bytes used
size_t mean_layout(const altgdmin_ctx* c, char* base, Aux* a) {
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = al256(off + b);
    return base ? base + o : nullptr;
  };
  Aux t{};
  t.v0 = reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)c->n));
  t.v1 = reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)c->n));
  t.v2 = reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)c->n));
  t.ci = reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)c->p.nc * c->n));
  t.part = reinterpret_cast<double*>(take(sizeof(double) * MRI_NB));
  t.cg = reinterpret_cast<CgState*>(take(sizeof(CgState)));
  if (a) *a = t;
  return off;
}

// the device error, if any, after a synchronisation
altgdmin_status sync_status(altgdmin_ctx* c) {
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ALTGDMIN_EHIP;
  int32_t err = 0;
  if (hipMemcpy(&err, &c->st()->err, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return ALTGDMIN_EHIP;
  return (altgdmin_status)err;
}

}  // namespace

extern "C" {

altgdmin_status altgdmin_aux_bytes(const altgdmin_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ALTGDMIN_EINVAL;
  *bytes = aux_layout(c, nullptr, nullptr);
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_mean(altgdmin_ctx* c, double tol, int32_t maxit, void* d_zbar, void* d_aux,
                              int32_t* h_iters) {
  if (!c || !d_zbar || !aux_ok(d_aux) || maxit < 0 || !(tol >= 0.0) || !isfinite(tol)) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  Aux a;
  aux_layout(c, static_cast<char*>(d_aux), &a);
  HIPCHK(mean_seq(c, tol, maxit, static_cast<float2*>(d_zbar), a));
  if (h_iters) {
    const altgdmin_status e = sync_status(c);
    HIPCHK(hipMemcpy(h_iters, &a.cg->iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (e != ALTGDMIN_OK) return e;
  }
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_mean_noalloc(altgdmin_ctx* c, double tol, int32_t maxit, void* d_zbar, int32_t* h_iters) {
  if (!c || !d_zbar || maxit < 0 || !(tol >= 0.0) || !isfinite(tol)) return ALTGDMIN_EINVAL;
  if (mean_layout(c, nullptr, nullptr) > kMeanScratchBytes) return ALTGDMIN_ESCRATCH;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  void* base = nullptr;
  const altgdmin_status s = scratch_address(&base);
  if (s != ALTGDMIN_OK) return s;
  Aux a;
  mean_layout(c, static_cast<char*>(base), &a);
  HIPCHK(mean_seq(c, tol, maxit, static_cast<float2*>(d_zbar), a));
  if (h_iters) {
    const altgdmin_status e = sync_status(c);
    HIPCHK(hipMemcpy(h_iters, &a.cg->iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (e != ALTGDMIN_OK) return e;
  }
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_residual(altgdmin_ctx* c, const void* d_zbar, const void* d_X, void* d_yres, void* d_aux) {
  if (!c || !d_yres || !aux_ok(d_aux)) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  Aux a;
  aux_layout(c, static_cast<char*>(d_aux), &a);
  hipStream_t s = c->stream;
  const long nq = (long)c->n * p.q;
  hipLaunchKernelGGL(k_form_z, dim3(grid_for(nq)), dim3(256), 0, s, static_cast<const float2*>(d_X),
                     static_cast<const float2*>(d_zbar), (long)c->n, p.q, a.v0, c->st());
  HIPCHK(hipGetLastError());
  float2* Y = static_cast<float2*>(d_yres);
  HIPCHK(ag_host::forward_op(c, a.v0, Y));
  const long ys = (long)p.q * p.nc * p.m_max;
  hipLaunchKernelGGL(k_sub_from, dim3(grid_for(ys)), dim3(256), 0, s, c->y, Y, c->m_k, p.nc, p.m_max, p.q, c->st());
  return map_hip(hipGetLastError());
}

altgdmin_status altgdmin_mec_cgls(altgdmin_ctx* c, const void* d_yres, int32_t iters, double tol, void* d_E,
                                  void* d_aux) {
  if (!c || !d_yres || !d_E || !aux_ok(d_aux) || iters < 0 || !(tol >= 0.0)) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  Aux a;
  aux_layout(c, static_cast<char*>(d_aux), &a);
  hipStream_t s = c->stream;
  DevState* st = c->st();
  const long n = c->n, nq = n * p.q, ylen = (long)p.nc * p.m_max, ys = ylen * p.q;
  float2* E = static_cast<float2*>(d_E);
  float2 *sv = a.v0, *pv = a.v1, *r = a.y0, *qv = a.y1;
  // r = yres on the valid samples (0 on the padding), s = A^H r, p = s
  hipLaunchKernelGGL(k_zero2, dim3(grid_for(nq)), dim3(256), 0, s, E, nq);
  hipLaunchKernelGGL(k_zero2, dim3(grid_for(ys)), dim3(256), 0, s, r, ys);
  hipLaunchKernelGGL(k_sub_from, dim3(grid_for(ys)), dim3(256), 0, s, static_cast<const float2*>(d_yres), r, c->m_k,
                     p.nc, p.m_max, p.q, st);
  HIPCHK(hipGetLastError());
  HIPCHK(ag_host::adjoint_op(c, r, sv, 0, 0));
  hipLaunchKernelGGL(k_copy2, dim3(grid_for(nq)), dim3(256), 0, s, sv, pv, nq);
  HIPCHK(frame_norms(c, sv, n, a.part));
  hipLaunchKernelGGL(k_frames_cg, dim3(1), dim3(128), 0, s, a.part, MRI_NBF, p.q, 0, tol, a.fc, st);
  HIPCHK(hipGetLastError());
  for (int it = 0; it < iters; ++it) {
    HIPCHK(ag_host::forward_op(c, pv, qv));
    HIPCHK(frame_norms(c, qv, ylen, a.part));
    hipLaunchKernelGGL(k_frames_cg, dim3(1), dim3(128), 0, s, a.part, MRI_NBF, p.q, 1, tol, a.fc, st);
    hipLaunchKernelGGL(k_frames_axpy, dim3(MRI_NBF, p.q), dim3(256), 0, s, E, pv, n, a.fc, 1, st);
    hipLaunchKernelGGL(k_frames_axpy, dim3(MRI_NBF, p.q), dim3(256), 0, s, r, qv, ylen, a.fc, -1, st);
    HIPCHK(hipGetLastError());
    HIPCHK(ag_host::adjoint_op(c, r, sv, 0, 0));
    HIPCHK(frame_norms(c, sv, n, a.part));
    hipLaunchKernelGGL(k_frames_cg, dim3(1), dim3(128), 0, s, a.part, MRI_NBF, p.q, 2, tol, a.fc, st);
    hipLaunchKernelGGL(k_frames_pupdate, dim3(MRI_NBF, p.q), dim3(256), 0, s, pv, sv, n, a.fc, st);
    HIPCHK(hipGetLastError());
  }
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_mec_ista(altgdmin_ctx* c, const void* d_yres, int32_t max_iter, double omega_frac,
                                  double tol, void* d_E, void* d_aux, int32_t* h_iters) {
  if (!c || !d_yres || !d_E || !aux_ok(d_aux) || max_iter < 0 || !(omega_frac >= 0.0) || !(tol >= 0.0))
    return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  Aux a;
  aux_layout(c, static_cast<char*>(d_aux), &a);
  hipStream_t s = c->stream;
  DevState* st = c->st();
  const long n = c->n, nq = n * p.q, ys = (long)p.q * p.nc * p.m_max;
  float2* E = static_cast<float2*>(d_E);
  const float2* yres = static_cast<const float2*>(d_yres);
  hipLaunchKernelGGL(k_ista_reset, dim3(1), dim3(1), 0, s, a.is);
  hipLaunchKernelGGL(k_zero2, dim3(grid_for(nq)), dim3(256), 0, s, E, nq);
  HIPCHK(hipGetLastError());
  float2* M[2] = {a.v1, a.v2};
  for (int t = 0; t < max_iter; ++t) {
    // V = E + A^H(yres - A(E)), M_t = F_t(V)
    HIPCHK(ag_host::forward_op(c, E, a.y0));
    hipLaunchKernelGGL(k_sub_from, dim3(grid_for(ys)), dim3(256), 0, s, yres, a.y0, c->m_k, p.nc, p.m_max, p.q, st);
    HIPCHK(hipGetLastError());
    HIPCHK(ag_host::adjoint_op(c, a.y0, a.v0, 0, 0));
    hipLaunchKernelGGL(k_add, dim3(grid_for(nq)), dim3(256), 0, s, a.v0, E, nq, st);
    float2* Mc = M[t & 1];
    HIPCHK(launch_tdft(a.v0, Mc, n, p.q, false, false, a.is, st, s));
    if (t == 0)
      hipLaunchKernelGGL(k_absmax_parts, dim3(MRI_NB), dim3(256), 0, s, Mc, nq, a.part, a.is, st);
    else
      hipLaunchKernelGGL(k_change_parts, dim3(MRI_NB), dim3(256), 0, s, Mc, M[(t + 1) & 1], nq, a.part, a.is, st);
    hipLaunchKernelGGL(k_ista_step, dim3(1), dim3(1), 0, s, a.part, MRI_NB, t, omega_frac, tol, a.is, st);
    HIPCHK(hipGetLastError());
    // E_{t+1} = F_t^{-1}(SThr_omega(M_t))
    HIPCHK(launch_tdft(Mc, E, n, p.q, true, true, a.is, st, s));
    hipLaunchKernelGGL(k_ista_commit, dim3(1), dim3(1), 0, s, a.is, st);
    HIPCHK(hipGetLastError());
  }
  if (h_iters) {
    const altgdmin_status e = sync_status(c);
    HIPCHK(hipMemcpy(h_iters, &a.is->iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (e != ALTGDMIN_OK) return e;
  }
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_expand(altgdmin_ctx* c, const void* d_U, const void* d_B, const void* d_zbar,
                                const void* d_E, void* d_Z) {
  if (!c || !d_Z || (!d_U) != (!d_B)) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  const long nq = (long)c->n * c->p.q;
  hipLaunchKernelGGL(k_expand, dim3(grid_for(nq)), dim3(256), 0, c->stream, static_cast<const float2*>(d_U),
                     static_cast<const float2*>(d_B), static_cast<const float2*>(d_zbar),
                     static_cast<const float2*>(d_E), (long)c->n, c->p.q, c->p.r, static_cast<float2*>(d_Z), c->st());
  return map_hip(hipGetLastError());
}

altgdmin_status altgdmin_rank_energy(altgdmin_ctx* c, int32_t r_cap, double* h_sigma2, void* d_aux) {
  if (!c || !h_sigma2 || !aux_ok(d_aux) || r_cap < 1 || r_cap > 16) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  if (r_cap > c->p.q) return ALTGDMIN_EINVAL;
  Aux a;
  aux_layout(c, static_cast<char*>(d_aux), &a);
  HIPCHK(ag_host::spectral_eig(c, r_cap, a.lam));
  const altgdmin_status e = sync_status(c);
  if (e != ALTGDMIN_OK) return e;
  HIPCHK(hipMemcpy(h_sigma2, a.lam, sizeof(double) * r_cap, hipMemcpyDeviceToHost));
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_auto_rank(altgdmin_ctx* c, double b_percent, int32_t* h_rank, int32_t* h_rcap,
                                   void* d_aux) {
  if (!c || !h_rank || !aux_ok(d_aux) || !(b_percent > 0.0) || !(b_percent <= 100.0)) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  std::vector<int32_t> mk(p.q);
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(mk.data(), c->m_k, sizeof(int32_t) * p.q, hipMemcpyDeviceToHost));
  const long mmin = *std::min_element(mk.begin(), mk.end());
  const long lim = std::min<long>(std::min<long>(c->n, p.q), (long)p.nc * mmin);
  const int r_cap = (int)std::max(1L, std::min(16L, lim / 10));
  double e2[16];
  const altgdmin_status st = altgdmin_rank_energy(c, r_cap, e2, d_aux);
  if (st != ALTGDMIN_OK) return st;
  double tot = 0.0;
  for (int j = 0; j < r_cap; ++j) tot += e2[j];
  const double target = b_percent / 100.0 * tot;
  int r = r_cap;
  double acc = 0.0;
  for (int j = 0; j < r_cap; ++j) {
    acc += e2[j];
    if (acc >= target) {
      r = j + 1;
      break;
    }
  }
  *h_rank = r;
  if (h_rcap) *h_rcap = r_cap;
  return ALTGDMIN_OK;
}

}  // extern "C"
