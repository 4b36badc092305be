// Transform kernels: batched 1D DFTs along x (contiguous rows) and along y
// (image columns), with the coil weighting, the sampling selection and the
// conjugate-coil combine fused into their loads and stores.
//
// The 2D DFT of the measurement model (Sec. II-A) is separable, F = F_y F_x.
// For 1D Cartesian masks every sampled line is complete along kx, so the
// kx half moves to a one-time pass over the data and each iteration needs
// only the y half, restricted on output to the sampled lines.  For general
// masks both halves run.
#include "kernels.hpp"

namespace ag {

// ---------------------------------------------------------------------------
// twiddle table: tw[t] = exp(-2 pi i t / N), from a double-precision sincospi
// ---------------------------------------------------------------------------
__global__ void k_twiddle(float2* tw, int N) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) {
    double s, c;
    sincospi(2.0 * (double)t / (double)N, &s, &c);
    tw[t] = make_float2((float)c, (float)(-s));
  }
}

// ---------------------------------------------------------------------------
// rows: FFT along x of TR rows of length N per workgroup.
// Row rho of the batch lives at src + rho*N.  With m_k != null the rows are
// the padded measurement lines rho = (k*nc + c)*lmax + l, valid when
// l < m_k[k]/N; invalid rows are written as zeros.  trunc: zero every input
// sample with |v|^2 > gamma (state) before the transform.
// ---------------------------------------------------------------------------
template <int N, int TR, bool INV>
__global__ __launch_bounds__(AG_NT) void k_rows(RowArgs a) {
  __shared__ float2 s[N * TR];
  const int tid = threadIdx.x;
  const long rho0 = (long)blockIdx.x * TR;
  if (halted(a.st, a.check_halt)) return;
  const double gamma = a.trunc ? a.st->gamma : 0.0;
  int n_cut = 0;
  for (int g = tid; g < N * TR; g += AG_NT) {
    const int t = g / N, e = g % N;
    const long rho = rho0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (rho < a.nrows && row_valid(a, rho, N)) {
      v = a.src[rho * N + e];
      if (a.trunc) {
        double m2 = (double)v.x * v.x + (double)v.y * v.y;
        if (m2 > gamma) {
          v = make_float2(0.f, 0.f);
          ++n_cut;
        }
      }
    }
    s[e * TR + t] = v;
  }
  if (n_cut && a.trunc_count) atomicAdd(a.trunc_count, n_cut);
  __syncthreads();
  fft_lds<N, TR, AG_NT, INV>(s, a.tw);
  for (int g = tid; g < N * TR; g += AG_NT) {
    const int t = g / N, e = g % N;
    const long rho = rho0 + t;
    if (rho < a.nrows) {
      float2 v = row_valid(a, rho, N) ? cscale(s[e * TR + t], a.scale) : make_float2(0.f, 0.f);
      a.dst[rho * N + e] = v;
    }
  }
}

// the same, register-fed (64 <= N <= 256): each thread's rows are loaded straight
// into the first radix pass (clamped rows, invalid ones zeroed after the
// load) and the last pass is stored from registers
template <int N, int TR, bool INV>
__global__ __launch_bounds__(AG_NT) void k_rows_regs(RowArgs a) {
  using GM = FftGeom<N, TR, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  __shared__ float2 s[FftPlan<N>::P > 1 ? N * TR : 1];
  __shared__ float2 s_tw[N];
  const int tid = threadIdx.x;
  const long rho0 = (long)blockIdx.x * TR;
  float2 v0[IT0][R0];
  bool okr[IT0];
#pragma unroll
  for (int it = 0; it < IT0; ++it) {
    const int g0 = tid + it * AG_NT, gg = GM::in_ok(g0) ? g0 : 0;
    const long rho = rho0 + gg % TR, rc = min(rho, a.nrows - 1);
    okr[it] = GM::in_ok(g0) && rho < a.nrows && row_valid(a, rc, N);
#pragma unroll
    for (int q = 0; q < R0; ++q) v0[it][q] = a.src[rc * N + GM::in_row(gg, q)];
  }
  for (int e = tid; e < N; e += AG_NT) {
    const float2 w = a.tw[e];
    s_tw[e] = INV ? make_float2(w.x, -w.y) : w;  // the inverse takes the conjugated table
  }
  if (halted(a.st, a.check_halt)) return;
  const double gamma = a.trunc ? a.st->gamma : 0.0;
  int n_cut = 0;
#pragma unroll
  for (int it = 0; it < IT0; ++it)
#pragma unroll
    for (int q = 0; q < R0; ++q) {
      const float2 v = v0[it][q];
      const bool cut = a.trunc && okr[it] && ((double)v.x * v.x + (double)v.y * v.y > gamma);
      n_cut += cut;
      if (!okr[it] || cut) v0[it][q] = make_float2(0.f, 0.f);
    }
  if (n_cut && a.trunc_count) atomicAdd(a.trunc_count, n_cut);
  __syncthreads();
  float2 vo[ITL][RL];
  fft_regs<N, TR, AG_NT, INV>(v0, vo, s, s_tw);
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int g = tid + it * AG_NT;
    const long rho = rho0 + g % TR;
    if (GM::out_ok(g) && rho < a.nrows) {
      const bool valid = row_valid(a, rho, N);
#pragma unroll
      for (int q = 0; q < RL; ++q)
        a.dst[rho * N + GM::out_row(g, q)] = valid ? cscale(vo[it][q], a.scale) : make_float2(0.f, 0.f);
    }
  }
}

// ---------------------------------------------------------------------------
// forward column transform: dst rows = F_y (s_c o src_img) restricted to a
// row list.  Grid (nx/TX, n_img, nc).
// ---------------------------------------------------------------------------
template <int N, int TX>
__global__ __launch_bounds__(AG_NT) void k_cols_fwd(ColFwdArgs a) {
  __shared__ float2 s[N * TX];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, img = blockIdx.y, c = blockIdx.z;
  if (halted(a.st, a.check_halt)) return;
  const float2* src = a.src + (long)img * a.src_img_stride;
  const float2* coil = a.coils + (long)c * a.n;
  {
    constexpr int IT = (N * TX + AG_NT - 1) / AG_NT;
    float2 cv[IT], uv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < N * TX) {
        const long p = (long)(g / TX) * a.nx + x0 + (g % TX);
        cv[it] = coil[p];
        uv[it] = src[p];
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < N * TX) s[g] = cmul(cv[it], uv[it]);
    }
  }
  __syncthreads();
  fft_lds<N, TX, AG_NT, false>(s, a.tw);
  int n_rows;
  const int32_t* rows = nullptr;
  if (a.m_k) {
    n_rows = a.m_k[img] / a.nx;
    rows = a.rows + (long)img * a.rows_img_stride;
  } else if (a.n_rows_ptr) {
    n_rows = *a.n_rows_ptr;
    rows = a.rows;
  } else {
    n_rows = N;
  }
  float2* dst = a.dst + (long)c * a.dst_c_stride + (long)img * a.dst_img_stride;
  for (int g = tid; g < n_rows * TX; g += AG_NT) {
    const int u = g / TX, col = g % TX;
    const int ky = rows ? rows[u] : u;
    dst[(long)u * a.nx + x0 + col] = cscale(s[ky * TX + col], a.scale);
  }
  if (a.zero_pad_rows > 0) {  // padding lines of a measurement layout
    for (int g = tid; g < (a.zero_pad_rows - n_rows) * TX; g += AG_NT) {
      const int u = n_rows + g / TX, col = g % TX;
      dst[(long)u * a.nx + x0 + col] = make_float2(0.f, 0.f);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint column transform with the coil combine:
//   dst_img = scale_img * sum_c conj(s_c) o F_y^H (rows of src_{c,img}
//             scattered onto their ky, zeros elsewhere).
// Grid (nx/TX, n_img).
// ---------------------------------------------------------------------------
template <int N, int TX>
__global__ __launch_bounds__(AG_NT) void k_cols_adj(ColAdjArgs a) {
  __shared__ float2 s[N * TX];
  constexpr int IT = (N * TX + AG_NT - 1) / AG_NT;
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, img = blockIdx.y;
  if (halted(a.st, a.check_halt)) return;
  int n_rows;
  const int32_t* rows = nullptr;
  if (a.m_k_rows) {
    n_rows = a.m_k_rows[img] / a.nx;
    rows = a.rows + (long)img * a.rows_img_stride;
  } else if (a.n_rows_ptr) {
    n_rows = *a.n_rows_ptr;
    rows = a.rows;
  } else {
    n_rows = N;
  }
  const bool full = (rows == nullptr);
  float2 acc[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) acc[it] = make_float2(0.f, 0.f);
  const int cb = blockIdx.z * a.cgs, ce = min(a.nc, cb + a.cgs);
  // a coil's sampled rows and its map, loaded one coil ahead so that the
  // loads overlap the previous coil's transform; every load is issued from
  // a valid (clamped) address and masked afterwards (a load under a branch
  // would be waited for on its own)
  float2 v[IT], cw[IT];
  int rv[IT];  // the row table's entries (ky of each sampled row), used once the data are staged
  // (with every row present the row table is not read: its stand-in is the
  // coil maps, readable at any u < N, and the value is discarded)
  const int32_t* const rtab = full ? reinterpret_cast<const int32_t*>(a.coils) : rows;
  auto fetch = [&](int c) {
    const float2* src = a.src + (long)c * a.src_c_stride + (long)img * a.src_img_stride;
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int g = tid + j * AG_NT;
      const int gc = g < n_rows * TX ? g : 0, u = gc / TX, col = gc % TX;
      rv[j] = rtab[u];
      v[j] = src[(long)u * a.nx + x0 + col];
      const int gm = min(g, N * TX - 1);
      cw[j] = coil[(long)(gm / TX) * a.nx + x0 + gm % TX];
    }
  };
  if (cb < ce) fetch(cb);
  for (int c = cb; c < ce; ++c) {
    if (!full) {
      for (int g = tid; g < N * TX; g += AG_NT) s[g] = make_float2(0.f, 0.f);
      __syncthreads();
    }
    float2 cwc[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int g = tid + j * AG_NT;
      if (g < n_rows * TX) s[(full ? g / TX : rv[j]) * TX + g % TX] = v[j];
      cwc[j] = cw[j];
    }
    __syncthreads();
    if (c + 1 < ce) fetch(c + 1);
    fft_lds<N, TX, AG_NT, true>(s, a.tw);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < N * TX) acc[it] = cadd(acc[it], cjmul(cwc[it], s[g]));
    }
    __syncthreads();
  }
  float sc = a.scale;
  if (a.m_k_scale) sc *= (float)(1.0 / sqrt((double)a.m_k_scale[img] * a.st->mbar));
  float2* dst = a.dst + (long)img * a.dst_img_stride + (long)blockIdx.z * a.dst_part_stride;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * AG_NT;
    if (g >= N * TX) break;
    const int y = g / TX, col = g % TX;
    const long p = (long)y * a.nx + x0 + col;
    float2 v = cscale(acc[it], sc);
    if (a.accumulate) v = cadd(dst[p], v);
    dst[p] = v;
  }
}

// ---------------------------------------------------------------------------
// the column adjoint with the coil combine for 1D line masks, register-fed:
// one workgroup per (CT-column tile, image), NG groups of 256 threads, group
// g transforming coils g, g + NG, ...; the image's sampled rows enter the
// first radix pass straight from registers through an inverse row map in
// LDS (k-space row -> the image's line holding it, -1 for a zero row), the
// coil-weighted sum is taken on the last pass's registers and the groups'
// sums meet in LDS at the end; the next coil's rows are loaded during the
// current transform.  Grid (nx / CT, images).
// ---------------------------------------------------------------------------
template <int N, int CT, int NG>
__global__ __launch_bounds__(AG_NT * NG) void k_cols_adj_lines(ColAdjArgs a) {
  using GM = FftGeom<N, CT, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  static_assert(FftPlan<N>::P > 1, "the groups' sums meet in the transform's LDS tiles");
  __shared__ float2 s[NG][N * CT];
  __shared__ float2 s_tw[N];
  __shared__ int s_li[N];
  const int tid = threadIdx.x, grp = tid / AG_NT, lt = tid % AG_NT;
  const int x0 = blockIdx.x * CT, img = blockIdx.y;
  if (halted(a.st, a.check_halt)) return;  // (a mask that failed its checks at bind sets err)
  const int n_rows = a.m_k_rows[img] / a.nx;
  const int32_t* rows = a.rows + (long)img * a.rows_img_stride;
  for (int e = tid; e < N; e += AG_NT * NG) {
    const float2 w = a.tw[e];
    s_tw[e] = make_float2(w.x, -w.y);  // the forward table conjugated: the inverse twiddles
    s_li[e] = -1;
  }
  __syncthreads();
  for (int l = tid; l < n_rows; l += AG_NT * NG) s_li[min(max(rows[l], 0), N - 1)] = l;  // an image's rows are distinct
  __syncthreads();
  float2 acc[ITL][RL];
#pragma unroll
  for (int it = 0; it < ITL; ++it)
#pragma unroll
    for (int q = 0; q < RL; ++q) acc[it][q] = make_float2(0.f, 0.f);
  int li[IT0][R0];  // this thread's input rows: the line holding each, -1 for a zero row
#pragma unroll
  for (int it = 0; it < IT0; ++it)
#pragma unroll
    for (int q = 0; q < R0; ++q) {
      const int g = lt + it * AG_NT;
      li[it][q] = GM::in_ok(g) ? s_li[GM::in_row(g, q)] : -1;
    }
  const float2* const src0 = a.src + (long)img * a.src_img_stride + x0;
  float2 kv[IT0][R0];
  auto fetch = [&](int c) {  // valid addresses for every lane; zero rows selected afterwards
    const float2* src = src0 + (long)min(c, a.nc - 1) * a.src_c_stride;
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
      const int col = (lt + it * AG_NT) % CT;
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const float2 v = src[(long)max(li[it][q], 0) * a.nx + col];
        kv[it][q] = li[it][q] >= 0 ? v : make_float2(0.f, 0.f);
      }
    }
  };
  fetch(grp);
  // every group runs the same number of rounds (the transforms' barriers are
  // the workgroup's); a group past the last coil transforms a copy of it and
  // does not add it
  for (int c0 = 0; c0 < a.nc; c0 += NG) {
    const int c = c0 + grp;
    float2 v0[IT0][R0], vo[ITL][RL];
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int q = 0; q < R0; ++q) v0[it][q] = kv[it][q];
    if (c0 + NG < a.nc) fetch(c + NG);
    fft_regs<N, CT, AG_NT, true>(v0, vo, s[grp], s_tw);
    // the coil values at the output rows come from the cache (every image
    // reads the same maps); loading them one coil ahead cost more in
    // registers than it saved
    if (c < a.nc) {
      const float2* coil = a.coils + (long)c * a.n + x0;
#pragma unroll
      for (int it = 0; it < ITL; ++it) {
        const int g = lt + it * AG_NT, col = g % CT;
        if (GM::out_ok(g)) {
#pragma unroll
          for (int q = 0; q < RL; ++q)
            acc[it][q] = cjfma(acc[it][q], coil[(long)GM::out_row(g, q) * a.nx + col], vo[it][q]);
        }
      }
    }
  }
  // the groups' sums: groups 1.. leave theirs in their (now free) LDS tiles
  if constexpr (NG > 1) {
    if (grp > 0) {
#pragma unroll
      for (int it = 0; it < ITL; ++it)
#pragma unroll
        for (int q = 0; q < RL; ++q) s[grp][(it * RL + q) * AG_NT + lt] = acc[it][q];
    }
    __syncthreads();
    if (grp > 0) return;
#pragma unroll
    for (int g2 = 1; g2 < NG; ++g2)
#pragma unroll
      for (int it = 0; it < ITL; ++it)
#pragma unroll
        for (int q = 0; q < RL; ++q) acc[it][q] = cadd(acc[it][q], s[g2][(it * RL + q) * AG_NT + lt]);
  }
  float sc = a.scale;
  if (a.m_k_scale) sc *= (float)(1.0 / sqrt((double)a.m_k_scale[img] * a.st->mbar));
  float2* dst = a.dst + (long)img * a.dst_img_stride + x0;
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int g = lt + it * AG_NT, col = g % CT;
    if (GM::out_ok(g)) {
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        const long p = (long)GM::out_row(g, q) * a.nx + col;
        float2 v = cscale(acc[it][q], sc);
        if (a.accumulate) v = cadd(dst[p], v);
        dst[p] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// general masks: gather the frame's samples from full k-space images, and
// the adjoint scatter (with optional truncation).
// ---------------------------------------------------------------------------
__global__ void k_gather(const float2* img, long img_stride_c, long img_stride_k, const int32_t* mask,
                         const int32_t* m_k, int m_max, int nc, int k0, float2* y, const DevState* st) {
  if (st->err) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int kk = blockIdx.y, c = blockIdx.z, k = k0 + kk;
  if (i >= m_max) return;
  float2 v = make_float2(0.f, 0.f);
  if (i < m_k[k]) v = img[c * img_stride_c + kk * img_stride_k + mask[(long)k * m_max + i]];
  y[((long)k * nc + c) * m_max + i] = v;
}

__global__ void k_scatter(const float2* y, const int32_t* mask, const int32_t* m_k, int m_max, int nc,
                          int k0, float2* img, long img_stride_c, long img_stride_k, const DevState* st,
                          int trunc, int32_t* trunc_count) {
  if (st->err) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int kk = blockIdx.y, c = blockIdx.z, k = k0 + kk;
  if (i >= m_k[k]) return;
  float2 v = y[((long)k * nc + c) * m_max + i];
  if (trunc) {
    double m2 = (double)v.x * v.x + (double)v.y * v.y;
    if (m2 > st->gamma) {
      v = make_float2(0.f, 0.f);
      if (trunc_count) atomicAdd(trunc_count, 1);
    }
  }
  img[c * img_stride_c + kk * img_stride_k + mask[(long)k * m_max + i]] = v;
}

__global__ void k_zero(float2* p, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {  // 16-byte stores: two values per lane
    float4* p4 = reinterpret_cast<float4*>(p);
    for (long j = i; j < n / 2; j += stride) p4[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i == 0 && (n & 1)) p[n - 1] = make_float2(0.f, 0.f);
    return;
  }
  for (; i < n; i += stride) p[i] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// host-side dispatch over the transform length
// ---------------------------------------------------------------------------
template <int N>
static hipError_t launch_rows_n(const RowArgs& a, bool inv, hipStream_t st) {
  constexpr int TR = ColTile<N>::TX;
  dim3 grid((unsigned)((a.nrows + TR - 1) / TR));
  if constexpr (N >= 64 && N <= 256) {  // the lengths the tests cover
    if (inv)
      hipLaunchKernelGGL((k_rows_regs<N, TR, true>), grid, dim3(AG_NT), 0, st, a);
    else
      hipLaunchKernelGGL((k_rows_regs<N, TR, false>), grid, dim3(AG_NT), 0, st, a);
  } else {
    if (inv)
      hipLaunchKernelGGL((k_rows<N, TR, true>), grid, dim3(AG_NT), 0, st, a);
    else
      hipLaunchKernelGGL((k_rows<N, TR, false>), grid, dim3(AG_NT), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_rows(int N, const RowArgs& a, bool inv, hipStream_t st) {
  if (a.nrows <= 0) return hipSuccess;
  switch (N) {
    case 8: return launch_rows_n<8>(a, inv, st);
    case 16: return launch_rows_n<16>(a, inv, st);
    case 32: return launch_rows_n<32>(a, inv, st);
    case 64: return launch_rows_n<64>(a, inv, st);
    case 128: return launch_rows_n<128>(a, inv, st);
    case 256: return launch_rows_n<256>(a, inv, st);
    case 512: return launch_rows_n<512>(a, inv, st);
  }
  return hipErrorInvalidValue;
}

int col_tile(int N, int nx) {
  int tx = (N >= 512) ? 8 : (N >= 256 ? 16 : 32);
  return tx < nx ? tx : nx;
}

// the adjoint transform runs half-width tiles: twice the workgroups
int col_tile_adj(int N, int nx) {
  int tx = col_tile(N, nx) / 2;
  return tx < 8 ? (nx < 8 ? nx : 8) : tx;
}

template <int N, int TX>
static hipError_t launch_cols_tx(const ColFwdArgs* f, const ColAdjArgs* d, int n_img, int nc, hipStream_t st) {
  if (f) {
    dim3 grid((unsigned)(f->nx / TX), (unsigned)n_img, (unsigned)nc);
    hipLaunchKernelGGL((k_cols_fwd<N, TX>), grid, dim3(AG_NT), 0, st, *f);
  } else {
    const int cgs = d->cgs > 0 ? d->cgs : d->nc;
    dim3 grid((unsigned)(d->nx / TX), (unsigned)n_img, (unsigned)((d->nc + cgs - 1) / cgs));
    ColAdjArgs dd = *d;
    dd.cgs = cgs;
    hipLaunchKernelGGL((k_cols_adj<N, TX>), grid, dim3(AG_NT), 0, st, dd);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t launch_cols_n(const ColFwdArgs* f, const ColAdjArgs* d, int nx, int n_img, int nc, hipStream_t st) {
  const int tx = f ? col_tile(N, nx) : col_tile_adj(N, nx);
  if constexpr (N <= 128) {
    if (tx == 32) return launch_cols_tx<N, 32>(f, d, n_img, nc, st);
  }
  if constexpr (N <= 256) {
    if (tx == 16) return launch_cols_tx<N, 16>(f, d, n_img, nc, st);
  }
  if (tx == 8) return launch_cols_tx<N, 8>(f, d, n_img, nc, st);
  return hipErrorInvalidValue;
}

constexpr int COLS_NG = 2;  // coil groups of the line back-projection's workgroup

hipError_t launch_cols(int N, const ColFwdArgs* f, const ColAdjArgs* d, int nx, int n_img, int nc,
                       hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  // line masks, every coil in one workgroup: the register-fed transform
  if (d && d->m_k_rows && (d->cgs <= 0 || d->cgs >= d->nc)) {
    // two groups of 256 threads, each over every other coil (four spill)
    if (N == 256 && nx % 16 == 0) {
      hipLaunchKernelGGL((k_cols_adj_lines<256, 16, COLS_NG>), dim3(nx / 16, n_img), dim3(AG_NT * COLS_NG), 0, st, *d);
      return hipGetLastError();
    }
    if (N == 128 && nx % 32 == 0) {
      hipLaunchKernelGGL((k_cols_adj_lines<128, 32, COLS_NG>), dim3(nx / 32, n_img), dim3(AG_NT * COLS_NG), 0, st, *d);
      return hipGetLastError();
    }
  }
  switch (N) {
    case 8: return launch_cols_n<8>(f, d, nx, n_img, nc, st);
    case 16: return launch_cols_n<16>(f, d, nx, n_img, nc, st);
    case 32: return launch_cols_n<32>(f, d, nx, n_img, nc, st);
    case 64: return launch_cols_n<64>(f, d, nx, n_img, nc, st);
    case 128: return launch_cols_n<128>(f, d, nx, n_img, nc, st);
    case 256: return launch_cols_n<256>(f, d, nx, n_img, nc, st);
    case 512: return launch_cols_n<512>(f, d, nx, n_img, nc, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace ag
