// The learned warm start: a 4-layer 3x3 CNN mapping the 2q back-projected
// planes of a sequence to an n x r complex matrix M (channel 2j = Re M[:, j],
// 2j + 1 = Im M[:, j]), its projection loss L = r - tr(G^-1 C C^H)
// (G = M^H M, C = M^H U_tgt), the backward pass and Adam.
//
// Convolutions are implicit GEMMs on the matrix cores with BF16 operands and
// FP32 accumulation (v_mfma_f32_16x16x32_bf16; activations, gradients and
// the packed weights stay FP32 in memory and are rounded to BF16 as they are
// staged in LDS):
//   forward      D[co][px] = sum_kappa Wp[kappa][co] X'[kappa][px],
//                kappa = tap*cin + ci (tap = 3 ty + tx), plus a bias row;
//   input grad   the same kernel on dY with the flipped, transposed weights,
//                times the ReLU mask of the layer below;
//   weight grad  D[co][kappa] = sum_px dY[co][px] X'[kappa][px], per band of
//                image rows, then a deterministic reduction.
// X'[kappa][px] is the input channel ci shifted by the tap (zero outside the
// image).  Activations are [b][c][H][W] FP32.  MFMA lane layout (16x16x32):
// lane l holds A[l%16][8(l/16)+e] and B[8(l/16)+e][l%16], e = 0..7; result
// register v holds D[4(l/16)+v][l%16].
#include "kernels_core.hpp"

namespace ag {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4v mfma_bf16(const bf8& a, const bf8& b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

#define CV_T 8     // output tile is CV_T x CV_T pixels
#define CV_CH 32   // input channels staged per chunk (one MFMA contraction)
#define CV_CHP 40  // BF16 pitch of a staged pixel's / weight row's channels (80 bytes: 16-byte aligned)

// ---------------------------------------------------------------------------
// pack one layer's weights: forward [kappa][32] (kappa = tap*cin + ci, bias
// row 9*cin, zero rows up to kp), input-gradient [kappa'][32] with
// kappa' = tap'*cout + co, tap' the flipped tap, columns ci
// ---------------------------------------------------------------------------
__global__ void k_cnn_pack(const float* __restrict__ Wl, int cin, int cout, int kp, int kpb, float* __restrict__ Wf,
                           float* __restrict__ Wb) {
  const float* bl = Wl + (long)cout * cin * 9;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)kp * 32; e += (long)gridDim.x * blockDim.x) {
    const int kap = (int)(e / 32), co = (int)(e % 32);
    float v = 0.f;
    if (co < cout) {
      if (kap < 9 * cin) {
        const int tap = kap / cin, ci = kap % cin;
        v = Wl[((long)co * cin + ci) * 9 + tap];
      } else if (kap == 9 * cin) {
        v = bl[co];
      }
    }
    Wf[e] = v;
  }
  if (Wb) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)kpb * 32; e += (long)gridDim.x * blockDim.x) {
      const int kap = (int)(e / 32), ci = (int)(e % 32);
      float v = 0.f;
      if (ci < cin && kap < 9 * cout) {
        const int tapf = kap / cout, co = kap % cout;
        v = Wl[((long)co * cin + ci) * 9 + (8 - tapf)];
      }
      Wb[e] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// convolution as implicit GEMM: grid (tiles of CV_T x CV_T, batch), 256
// threads; wave w computes tile rows 2w, 2w + 1 (16 pixels) for all output
// channels (<= 32).  Per chunk of 32 input channels the tile's inputs (with
// the halo) are staged as BF16 [pixel][channel] and the chunk's weights as
// BF16 [tap][co][channel]: one 16x16x32 product per tap and output tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a) {
  constexpr int NPX = (CV_T + 2) * (CV_T + 2);
  __shared__ __attribute__((aligned(16))) __bf16 xs[NPX * CV_CHP];
  __shared__ __attribute__((aligned(16))) __bf16 wsm[9 * 32 * CV_CHP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_x = a.W / CV_T;
  const int ty0 = (blockIdx.x / tiles_x) * CV_T, tx0 = (blockIdx.x % tiles_x) * CV_T;
  const int b = blockIdx.y;
  const long plane = (long)a.H * a.W;
  const float* Xb = a.X + (long)b * a.cin * plane;
  const int pl = lane & 15, kq = lane >> 4;
  const int py = 2 * wave + (pl >> 3), px = pl & 7;
  const int nct = (a.cout + 15) >> 4;
  f4v acc[2] = {f4v{0.f, 0.f, 0.f, 0.f}, f4v{0.f, 0.f, 0.f, 0.f}};
  for (int c0 = 0; c0 < a.cin; c0 += CV_CH) {
    // channels past cin stage as zeros, so that the matrix-core loop has no
    // predicate (a second output tile past cout is computed and not stored);
    // every load comes from a valid address and is masked afterwards
    const int nch = min(CV_CH, a.cin - c0);
    __syncthreads();
    for (int e = tid; e < NPX * 4; e += 256) {  // (pixel, channel octet)
      const int pix = e % NPX, j = e / NPX;
      const int rr = pix / (CV_T + 2), cc = pix % (CV_T + 2);
      const int gy = ty0 + rr - 1, gx = tx0 + cc - 1;
      const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
      const long off = in ? (long)gy * a.W + gx : 0;
      float f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = Xb[(long)(c0 + min(8 * j + q, nch - 1)) * plane + off];
      bf8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (__bf16)((in && 8 * j + q < nch) ? f[q] : 0.f);
      *reinterpret_cast<bf8*>(&xs[pix * CV_CHP + 8 * j]) = v;
    }
    for (int e = tid; e < 9 * 32 * 4; e += 256) {  // (tap, channel octet, co) from the rows [tap*cin + ci][32]
      const int co = e & 31, j = (e >> 5) & 3, tap = e >> 7;
      const float* wr = a.Wp + ((long)tap * a.cin + c0) * 32 + co;
      float f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = wr[(long)min(8 * j + q, nch - 1) * 32];
      bf8 w;
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = (__bf16)(8 * j + q < nch ? f[q] : 0.f);
      *reinterpret_cast<bf8*>(&wsm[(tap * 32 + co) * CV_CHP + 8 * j]) = w;
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      const bf8 bv = *reinterpret_cast<const bf8*>(&xs[((py + dy) * (CV_T + 2) + px + dx) * CV_CHP + 8 * kq]);
      const bf8 w0 = *reinterpret_cast<const bf8*>(&wsm[(tap * 32 + pl) * CV_CHP + 8 * kq]);
      const bf8 w1 = *reinterpret_cast<const bf8*>(&wsm[(tap * 32 + 16 + pl) * CV_CHP + 8 * kq]);
      acc[0] = mfma_bf16(w0, bv, acc[0]);
      acc[1] = mfma_bf16(w1, bv, acc[1]);
    }
  }
  const int oy = ty0 + py, ox = tx0 + px;
  float* Yb = a.Y + (long)b * a.cout * plane;
  const float* Mb = a.mask ? a.mask + (long)b * a.cout * plane : nullptr;
  const long kb = 9L * a.cin * 32;  // the bias row of the packed weights (FP32, added exactly)
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t < nct) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int co = 16 * t + 4 * kq + v;
        if (co < a.cout) {
          float y = acc[t][v];
          if (a.bias) y += a.Wp[kb + co];
          if (a.relu) y = fmaxf(y, 0.f);
          const long o = (long)co * plane + (long)oy * a.W + ox;
          if (Mb && !(Mb[o] > 0.f)) y = 0.f;
          Yb[o] = y;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: grid (row bands, batch, kappa groups), 256 threads.  A
// band is rows_per_band image rows (whole tiles); the workgroup stages every
// input channel of a tile (with its halo) and the tile's output gradient as
// BF16 and covers WG_KT kappa tiles of 16 (8 per wave), one 16x16x32 product
// per 32 pixels, writing its partial dWp[kappa][co] to
// part + ((b * bands + band) * kp + kappa) * 32 + co.
// ---------------------------------------------------------------------------
#define WG_KTW 8            // kappa tiles per wave
#define WG_KT (4 * WG_KTW)  // kappa tiles per workgroup
#define XS_STRIDE ((CV_T + 2) * (CV_T + 3))
#define DS_PITCH (CV_T * CV_T + 8)  // BF16 pitch of a channel's 64 pixels (16-byte aligned rows)
__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs a) {
  extern __shared__ __bf16 xsb[];  // [cin][CV_T + 2][CV_T + 3]
  __shared__ __attribute__((aligned(16))) __bf16 ds[32 * DS_PITCH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pl = lane & 15, kq = lane >> 4;
  const int b = blockIdx.y;
  const long plane = (long)a.H * a.W;
  const float* Xb = a.X + (long)b * a.cin * plane;
  const float* Db = a.dY + (long)b * a.cout * plane;
  const int tiles_x = a.W / CV_T;
  const int nkt = (9 * a.cin + 1 + 15) >> 4;  // kappa tiles incl. the bias row
  const int nct = (a.cout + 15) >> 4;
  const int kt0 = blockIdx.z * WG_KT;
  f4v acc[WG_KTW][2];
#pragma unroll
  for (int m = 0; m < WG_KTW; ++m) acc[m][0] = acc[m][1] = f4v{0.f, 0.f, 0.f, 0.f};
  // per kappa tile of this lane: channel and tap offset (or the bias row)
  int kci[WG_KTW], koff[WG_KTW];
#pragma unroll
  for (int m = 0; m < WG_KTW; ++m) {
    const int kap = 16 * (kt0 + wave + 4 * m) + pl;
    kci[m] = -1;
    koff[m] = 0;
    if (kap < 9 * a.cin) {
      const int tap = kap / a.cin;
      kci[m] = kap % a.cin;
      koff[m] = (tap / 3) * (CV_T + 3) + tap % 3;
    } else if (kap == 9 * a.cin) {
      kci[m] = -2;  // bias: input 1
    }
  }
  const __bf16 one = (__bf16)1.f, zero = (__bf16)0.f;
  const int row0 = blockIdx.x * a.rows_per_band;
  for (int tr = row0; tr < row0 + a.rows_per_band; tr += CV_T) {
    for (int tc = 0; tc < tiles_x; ++tc) {
      const int ty0 = tr, tx0 = tc * CV_T;
      __syncthreads();
      for (int e = tid; e < 32 * CV_T * CV_T; e += 256) {
        const int co = e / (CV_T * CV_T), p = e % (CV_T * CV_T);
        const float d = Db[(long)min(co, a.cout - 1) * plane + (long)(ty0 + p / CV_T) * a.W + tx0 + p % CV_T];
        ds[co * DS_PITCH + p] = (__bf16)(co < a.cout ? d : 0.f);
      }
      for (int e = tid; e < a.cin * (CV_T + 2) * (CV_T + 2); e += 256) {
        const int ci = e / ((CV_T + 2) * (CV_T + 2)), rem = e % ((CV_T + 2) * (CV_T + 2));
        const int rr = rem / (CV_T + 2), cc = rem % (CV_T + 2);
        const int gy = ty0 + rr - 1, gx = tx0 + cc - 1;
        const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        const float v = Xb[(long)ci * plane + (in ? (long)gy * a.W + gx : 0)];
        xsb[ci * XS_STRIDE + rr * (CV_T + 3) + cc] = (__bf16)(in ? v : 0.f);
      }
      __syncthreads();
#pragma unroll
      for (int k0 = 0; k0 < CV_T * CV_T; k0 += 32) {
        // pixels k0 + 8 kq + e: tile row (k0 / 8 + kq), columns e = 0..7
        const int prow = k0 / CV_T + kq;
        const bf8 a0 = *reinterpret_cast<const bf8*>(&ds[pl * DS_PITCH + k0 + 8 * kq]);
        const bf8 a1 = *reinterpret_cast<const bf8*>(&ds[(16 + pl) * DS_PITCH + k0 + 8 * kq]);
#pragma unroll
        for (int m = 0; m < WG_KTW; ++m) {
          if (kt0 + wave + 4 * m < nkt) {
            const int ci = kci[m];
            bf8 bv;
            if (ci >= 0) {
              const __bf16* xr = xsb + ci * XS_STRIDE + prow * (CV_T + 3) + koff[m];
#pragma unroll
              for (int q = 0; q < 8; ++q) bv[q] = xr[q];
            } else {
#pragma unroll
              for (int q = 0; q < 8; ++q) bv[q] = (ci == -2) ? one : zero;
            }
            acc[m][0] = mfma_bf16(a0, bv, acc[m][0]);
            if (nct > 1) acc[m][1] = mfma_bf16(a1, bv, acc[m][1]);
          }
        }
      }
    }
  }
  float* out = a.part + (long)(blockIdx.y * gridDim.x + blockIdx.x) * a.kp * 32;
#pragma unroll
  for (int m = 0; m < WG_KTW; ++m) {
    const int kt = kt0 + wave + 4 * m;
    if (kt < nkt) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int co = 16 * t + 4 * kq + v;
          const int kap = 16 * kt + pl;
          if (kap < a.kp) out[(long)kap * 32 + co] = acc[m][t][v];
        }
      }
    }
  }
}

// sum the weight-gradient partials into the flat parameter gradient (W then
// b of this layer), times scale
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nparts, int kp, int cin, int cout, float scale,
                               float* __restrict__ g) {
  const int total = cout * cin * 9 + cout;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    int kap, co;
    if (e < cout * cin * 9) {
      co = e / (cin * 9);
      const int rem = e % (cin * 9), ci = rem / 9, tap = rem % 9;
      kap = tap * cin + ci;
    } else {
      co = e - cout * cin * 9;
      kap = 9 * cin;
    }
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += part[((long)q * kp + kap) * 32 + co];
    g[e] = (float)(s * scale);
  }
}

// ---------------------------------------------------------------------------
// loss: Gram of [M U_tgt] per sequence (FP64 partials over pixel chunks),
// the r x r algebra, then the output-channel gradient
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_gram(LossArgs a) {
  __shared__ float2 s[64][33];
  const int tid = threadIdx.x, b = blockIdx.y, r = a.r, m = 2 * r;
  const int nout = m * (m + 1) / 2;
  const float* Yb = a.Y4 + (long)b * 2 * r * a.n;
  const float2* Ub = a.Ut + (long)b * r * a.n;
  double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  const long p0 = (long)blockIdx.x * a.chunk, p1 = min(a.n, p0 + a.chunk);
  for (long pb = p0; pb < p1; pb += 64) {
    const int np = (int)min((long)64, p1 - pb);
    __syncthreads();
    for (int e = tid; e < 64 * m; e += 256) {
      const int j = e / 64, pp = e % 64;
      float2 v = make_float2(0.f, 0.f);
      if (pp < np) {
        const long p = pb + pp;
        v = (j < r) ? make_float2(Yb[(long)(2 * j) * a.n + p], Yb[(long)(2 * j + 1) * a.n + p])
                    : Ub[(long)(j - r) * a.n + p];
      }
      s[pp][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int o = tid + 256 * t;
      if (o < nout) {
        int i, j;
        tri_index(o, m, i, j);
        for (int pp = 0; pp < np; ++pp) {
          const float2 x = s[pp][i], y = s[pp][j];  // conj(x) y
          acc[t].x += (double)x.x * y.x + (double)x.y * y.y;
          acc[t].y += (double)x.x * y.y - (double)x.y * y.x;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int o = tid + 256 * t;
    if (o < nout) a.part[((long)b * gridDim.x + blockIdx.x) * nout + o] = acc[t];
  }
}

// one thread per sequence does the r x r work (r <= 16)
__global__ void k_loss_small(LossArgs a) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int r = a.r, m = 2 * r, nout = m * (m + 1) / 2;
  double2 G[16][16], Cm[16][16], L[16][16], Gi[16][16], T[16][16];
  auto entry = [&](int i, int j) {  // (i <= j) entry of the Gram of [M U]
    double2 s = make_double2(0.0, 0.0);
    int o = 0;
    for (int ii = 0; ii < i; ++ii) o += m - ii;
    o += j - i;
    for (int q = 0; q < a.nchunks; ++q) s = dadd(s, a.part[((long)b * a.nchunks + q) * nout + o]);
    return s;
  };
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) {
      const double2 v = entry(i, j);
      G[i][j] = v;
      G[j][i] = dconj(v);
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) Cm[i][j] = entry(i, r + j);  // (M^H U)[i][j]
  double tr = 0.0;
  for (int i = 0; i < r; ++i) tr += G[i][i].x;
  // Cholesky G = L L^H (a tiny ridge keeps a rank-deficient M finite)
  const double ridge = 1e-12 * tr / r;
  for (int j = 0; j < r; ++j) {
    double d = G[j][j].x + ridge;
    for (int k = 0; k < j; ++k) d -= L[j][k].x * L[j][k].x + L[j][k].y * L[j][k].y;
    d = sqrt(fmax(d, 1e-300));
    L[j][j] = make_double2(d, 0.0);
    for (int i = j + 1; i < r; ++i) {
      double2 s2 = G[i][j];
      for (int k = 0; k < j; ++k) s2 = dsub(s2, dmul(L[i][k], dconj(L[j][k])));
      L[i][j] = make_double2(s2.x / d, s2.y / d);
    }
  }
  // Gi = G^-1 column by column: L z = e_c, L^H x = z
  for (int c = 0; c < r; ++c) {
    double2 z[16];
    for (int i = 0; i < r; ++i) {
      double2 s2 = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int k = 0; k < i; ++k) s2 = dsub(s2, dmul(L[i][k], z[k]));
      z[i] = make_double2(s2.x / L[i][i].x, s2.y / L[i][i].x);
    }
    for (int i = r - 1; i >= 0; --i) {
      double2 s2 = z[i];
      for (int k = i + 1; k < r; ++k) s2 = dsub(s2, dmul(dconj(L[k][i]), Gi[k][c]));
      Gi[i][c] = make_double2(s2.x / L[i][i].x, s2.y / L[i][i].x);
    }
  }
  // T = C C^H; loss r - tr(Gi T); P1 = C^H Gi; P2 = Gi T Gi
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double2 s2 = make_double2(0.0, 0.0);
      for (int k = 0; k < r; ++k) s2 = dadd(s2, dmul(Cm[i][k], dconj(Cm[j][k])));
      T[i][j] = s2;
    }
  double lt = 0.0;
  for (int i = 0; i < r; ++i)
    for (int k = 0; k < r; ++k) lt += dmul(Gi[i][k], T[k][i]).x;
  a.loss_b[b] = r - lt;
  double2* P1 = a.P + (long)b * 2 * r * r;
  double2* P2 = P1 + r * r;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double2 s1 = make_double2(0.0, 0.0);
      for (int k = 0; k < r; ++k) s1 = dadd(s1, dmul(dconj(Cm[k][i]), Gi[k][j]));
      P1[i * r + j] = s1;
    }
  double2 GT[16][16];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double2 s2 = make_double2(0.0, 0.0);
      for (int k = 0; k < r; ++k) s2 = dadd(s2, dmul(Gi[i][k], T[k][j]));
      GT[i][j] = s2;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double2 s2 = make_double2(0.0, 0.0);
      for (int k = 0; k < r; ++k) s2 = dadd(s2, dmul(GT[i][k], Gi[k][j]));
      P2[i * r + j] = s2;
    }
}

// dL/d conj(M) = M P2 - U P1; output-channel gradient (2 Re, 2 Im) * scale
__global__ void k_loss_grad(LossArgs a) {
  const int b = blockIdx.y, r = a.r;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const float* Yb = a.Y4 + (long)b * 2 * r * a.n;
  const float2* Ub = a.Ut + (long)b * r * a.n;
  const double2* P1 = a.P + (long)b * 2 * r * r;
  const double2* P2 = P1 + r * r;
  float* dY = a.dY4 + (long)b * 2 * r * a.n;
  double2 Mp[16], Up[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    Mp[i] = Up[i] = make_double2(0.0, 0.0);
    if (i < r) {
      Mp[i] = make_double2(Yb[(long)(2 * i) * a.n + p], Yb[(long)(2 * i + 1) * a.n + p]);
      const float2 u = Ub[(long)i * a.n + p];
      Up[i] = make_double2(u.x, u.y);
    }
  }
  for (int j = 0; j < r; ++j) {
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i < r) s = dadd(s, dsub(dmul(Mp[i], P2[i * r + j]), dmul(Up[i], P1[i * r + j])));
    dY[(long)(2 * j) * a.n + p] = (float)(2.0 * s.x * a.scale);
    dY[(long)(2 * j + 1) * a.n + p] = (float)(2.0 * s.y * a.scale);
  }
}

__global__ void k_loss_total(const double* loss_b, int batch, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < batch; ++b) s += loss_b[b];
  *out = s / batch;
}

// network output -> M, n x r column-major complex per sequence
__global__ void k_cnn_to_M(const float* Y4, int r, long n, int batch, float2* M) {
  const long total = (long)batch * r * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long b = e / ((long)r * n), rem = e % ((long)r * n);
    const int j = (int)(rem / n);
    const long p = rem % n;
    const float* Yb = Y4 + b * 2 * r * n;
    M[e] = make_float2(Yb[(long)(2 * j) * n + p], Yb[(long)(2 * j + 1) * n + p]);
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float c1, float c2, float eps) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_cnn_pack(const float* Wl, int cin, int cout, int kp, int kpb, float* Wf, float* Wb, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_pack, dim3(64), dim3(256), 0, s, Wl, cin, cout, kp, kpb, Wf, Wb);
  return hipGetLastError();
}

hipError_t launch_conv(const ConvArgs& a, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_conv_fwd, dim3((a.H / CV_T) * (a.W / CV_T), batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int bands, int batch, int nparam_layer, float* g, float scale,
                        hipStream_t s) {
  const int nkt = (9 * a.cin + 1 + 15) / 16;
  const size_t lds = sizeof(__bf16) * (size_t)a.cin * XS_STRIDE;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_wgrad, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_conv_wgrad, dim3(bands, batch, (nkt + WG_KT - 1) / WG_KT), dim3(256), lds, s, a);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nparam_layer + 255) / 256), dim3(256), 0, s, a.part, bands * batch, a.kp,
                     a.cin, a.cout, scale, g);
  return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, int batch, double* d_loss, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_gram, dim3(a.nchunks, batch), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_loss_small, dim3(batch), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)((a.n + 255) / 256), batch), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, a.loss_b, batch, d_loss);
  return hipGetLastError();
}

hipError_t launch_cnn_to_M(const float* Y4, int r, long n, int batch, float2* M, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_to_M, dim3(1024), dim3(256), 0, s, Y4, r, n, batch, M);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - pow(0.9, step)), c2 = (float)(1.0 - pow(0.999, step));
  hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, c1, c2, 1e-8f);
  return hipGetLastError();
}

// L1: 2q planes (Re, Im of column k of X = A^H(y)) divided by their RMS.
// Pass 1: FP64 partial sums of squares per workgroup; pass 2: every
// workgroup re-sums the partials and writes its share.
__global__ __launch_bounds__(256) void k_planes_sumsq(const float2* X, long total, double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const float2 v = X[e];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_planes_write(const float2* X, long n, int q, const double* partial,
                                                      int nparts, float* out) {
  __shared__ float s_inv;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += partial[i];
    const double rms = sqrt(s / (2.0 * q * n));
    s_inv = rms > 0.0 ? (float)(1.0 / rms) : 1.f;
  }
  __syncthreads();
  const float inv = s_inv;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < (long)q * n; e += (long)gridDim.x * 256) {
    const long k = e / n, p = e % n;
    const float2 v = X[e];
    out[(2 * k) * n + p] = v.x * inv;
    out[(2 * k + 1) * n + p] = v.y * inv;
  }
}

hipError_t launch_cnn_planes(const float2* X, long n, int q, double* partial, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_planes_sumsq, dim3(256), dim3(256), 0, s, X, n * q, partial);
  hipLaunchKernelGGL(k_planes_write, dim3(256), dim3(256), 0, s, X, n, q, partial, 256, out);
  return hipGetLastError();
}

}  // namespace ag
