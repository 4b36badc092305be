// Host side of the warm-start CNN: shapes, workspace layout and the order
// of the launches for the forward pass, the loss and backward pass, and Adam.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/wsinit.h"
#include "kernels_core.hpp"

using namespace ag;

struct wsinit_ctx {
  int nx, ny, q, r, width, layers, max_batch;
  long n;
  hipStream_t stream;
  struct Layer {
    int cin, cout, kp, kpb;
    long poff, nparam;
    size_t o_wf, o_wb;
  } L[4];
  int bands, rows_per_band, chunk, nchunks;
  size_t o_h[4], o_y4, o_dz[2], o_dy4, o_part, o_lpart, o_P, o_lossb, bytes;
  long nparams;
  template <typename T>
  T* at(void* ws, size_t off) const {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
  }
};

namespace {

#define WCHK(x)                                                   \
  do {                                                            \
    hipError_t e_ = (x);                                          \
    if (e_ != hipSuccess) return ALTGDMIN_EHIP;                   \
  } while (0)

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

altgdmin_status forward_layers(wsinit_ctx* h, const float* params, const float* in, int batch, void* ws) {
  for (int l = 0; l < 4; ++l) {
    const auto& Ly = h->L[l];
    WCHK(launch_cnn_pack(params + Ly.poff, Ly.cin, Ly.cout, Ly.kp, Ly.kpb, h->at<float>(ws, Ly.o_wf),
                         l > 0 ? h->at<float>(ws, Ly.o_wb) : nullptr, h->stream));
  }
  for (int l = 0; l < 4; ++l) {
    const auto& Ly = h->L[l];
    ConvArgs a{};
    a.X = l == 0 ? in : h->at<float>(ws, h->o_h[l]);
    a.Wp = h->at<float>(ws, Ly.o_wf);
    a.Y = l == 3 ? h->at<float>(ws, h->o_y4) : h->at<float>(ws, h->o_h[l + 1]);
    a.mask = nullptr;
    a.cin = Ly.cin;
    a.cout = Ly.cout;
    a.H = h->ny;
    a.W = h->nx;
    a.bias = 1;
    a.relu = l < 3;
    WCHK(launch_conv(a, batch, h->stream));
  }
  return ALTGDMIN_OK;
}

}  // namespace

extern "C" {

altgdmin_status wsinit_create(int32_t nx, int32_t ny, int32_t q, int32_t r, int32_t width, int32_t layers,
                              int32_t batch, void* stream, wsinit_ctx** out) {
  if (!out) return ALTGDMIN_EINVAL;
  *out = nullptr;
  if (nx < 8 || ny < 8 || nx > 512 || ny > 512 || nx % 8 || ny % 8) return ALTGDMIN_EINVAL;
  if (q < 1 || q > 128 || r < 1 || r > 16 || width < 4 || width > 32 || layers != 4) return ALTGDMIN_EINVAL;
  if (batch < 1 || batch > 64) return ALTGDMIN_EINVAL;
  wsinit_ctx* h = new (std::nothrow) wsinit_ctx();
  if (!h) return ALTGDMIN_EINVAL;
  h->nx = nx;
  h->ny = ny;
  h->q = q;
  h->r = r;
  h->width = width;
  h->layers = layers;
  h->max_batch = batch;
  h->n = (long)nx * ny;
  h->stream = static_cast<hipStream_t>(stream);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  long poff = 0;
  int max_kp = 0;
  for (int l = 0; l < 4; ++l) {
    auto& Ly = h->L[l];
    Ly.cin = l == 0 ? 2 * q : width;
    Ly.cout = l == 3 ? 2 * r : width;
    Ly.kp = (9 * Ly.cin + 1 + 15) / 16 * 16;
    Ly.kpb = 9 * Ly.cout;
    Ly.poff = poff;
    Ly.nparam = (long)Ly.cout * Ly.cin * 9 + Ly.cout;
    poff += Ly.nparam;
    Ly.o_wf = take(sizeof(float) * Ly.kp * 32);
    Ly.o_wb = take(sizeof(float) * Ly.kpb * 32);
    if (Ly.kp > max_kp) max_kp = Ly.kp;
  }
  h->nparams = poff;
  const size_t act = sizeof(float) * (size_t)batch * width * h->n;
  h->o_h[0] = 0;
  for (int l = 1; l < 4; ++l) h->o_h[l] = take(act);
  h->o_y4 = take(sizeof(float) * (size_t)batch * 2 * r * h->n);
  h->o_dz[0] = take(act);
  h->o_dz[1] = take(act);
  h->o_dy4 = take(sizeof(float) * (size_t)batch * 2 * r * h->n);
  h->rows_per_band = 8;
  h->bands = ny / 8;
  h->o_part = take(sizeof(float) * (size_t)batch * h->bands * max_kp * 32);
  h->chunk = 1024;
  h->nchunks = (int)((h->n + h->chunk - 1) / h->chunk);
  const int m = 2 * r;
  h->o_lpart = take(sizeof(double2) * (size_t)batch * h->nchunks * (m * (m + 1) / 2));
  h->o_P = take(sizeof(double2) * (size_t)batch * 2 * r * r);
  h->o_lossb = take(sizeof(double) * batch);
  h->bytes = off;
  *out = h;
  return ALTGDMIN_OK;
}

altgdmin_status wsinit_param_count(const wsinit_ctx* h, int64_t* count) {
  if (!h || !count) return ALTGDMIN_EINVAL;
  *count = h->nparams;
  return ALTGDMIN_OK;
}

altgdmin_status wsinit_workspace_bytes(const wsinit_ctx* h, size_t* bytes) {
  if (!h || !bytes) return ALTGDMIN_EINVAL;
  *bytes = h->bytes;
  return ALTGDMIN_OK;
}

altgdmin_status wsinit_forward(wsinit_ctx* h, const float* params, const float* in, int32_t batch, void* d_M,
                               void* ws) {
  if (!h || !params || !in || !d_M || !ws || !aligned(ws)) return ALTGDMIN_EINVAL;
  if (batch < 1 || batch > h->max_batch) return ALTGDMIN_EINVAL;
  const altgdmin_status st = forward_layers(h, params, in, batch, ws);
  if (st != ALTGDMIN_OK) return st;
  WCHK(launch_cnn_to_M(h->at<float>(ws, h->o_y4), h->r, h->n, batch, static_cast<float2*>(d_M), h->stream));
  return ALTGDMIN_OK;
}

altgdmin_status wsinit_loss_backward(wsinit_ctx* h, const float* params, const float* in, const void* d_Ut,
                                     int32_t batch, float* grads, double* d_loss, void* ws) {
  if (!h || !params || !in || !d_Ut || !grads || !d_loss || !ws || !aligned(ws)) return ALTGDMIN_EINVAL;
  if (batch < 1 || batch > h->max_batch) return ALTGDMIN_EINVAL;
  altgdmin_status st = forward_layers(h, params, in, batch, ws);
  if (st != ALTGDMIN_OK) return st;
  LossArgs la{};
  la.Y4 = h->at<float>(ws, h->o_y4);
  la.Ut = static_cast<const float2*>(d_Ut);
  la.part = h->at<double2>(ws, h->o_lpart);
  la.P = h->at<double2>(ws, h->o_P);
  la.loss_b = h->at<double>(ws, h->o_lossb);
  la.dY4 = h->at<float>(ws, h->o_dy4);
  la.n = h->n;
  la.chunk = h->chunk;
  la.r = h->r;
  la.nchunks = h->nchunks;
  la.scale = 1.0f / batch;
  WCHK(launch_loss(la, batch, d_loss, h->stream));
  // backward: dZ_3 = dY4; for each layer the weight gradient, then the
  // gradient at its input times the ReLU mask of that input
  const float* dz = h->at<float>(ws, h->o_dy4);
  int ping = 0;
  for (int l = 3; l >= 0; --l) {
    const auto& Ly = h->L[l];
    const float* X = l == 0 ? in : h->at<float>(ws, h->o_h[l]);
    WgradArgs wa{};
    wa.X = X;
    wa.dY = dz;
    wa.part = h->at<float>(ws, h->o_part);
    wa.cin = Ly.cin;
    wa.cout = Ly.cout;
    wa.H = h->ny;
    wa.W = h->nx;
    wa.kp = Ly.kp;
    wa.rows_per_band = h->rows_per_band;
    WCHK(launch_wgrad(wa, h->bands, batch, (int)Ly.nparam, grads + Ly.poff, 1.0f, h->stream));
    if (l > 0) {
      ConvArgs a{};
      a.X = dz;
      a.Wp = h->at<float>(ws, Ly.o_wb);
      float* dnext = h->at<float>(ws, h->o_dz[ping]);
      a.Y = dnext;
      a.mask = X;  // h_l = relu(z_{l-1})
      a.cin = Ly.cout;
      a.cout = Ly.cin;
      a.H = h->ny;
      a.W = h->nx;
      a.bias = 0;
      a.relu = 0;
      WCHK(launch_conv(a, batch, h->stream));
      dz = dnext;
      ping ^= 1;
    }
  }
  return ALTGDMIN_OK;
}

altgdmin_status wsinit_adam_step(wsinit_ctx* h, float* params, const float* grads, float* m, float* v, float lr,
                                 int32_t step) {
  if (!h || !params || !grads || !m || !v || step < 1 || !(lr > 0.f)) return ALTGDMIN_EINVAL;
  WCHK(launch_adam(params, grads, m, v, h->nparams, lr, step, h->stream));
  return ALTGDMIN_OK;
}

void wsinit_destroy(wsinit_ctx* h) { delete h; }

}  // extern "C"
