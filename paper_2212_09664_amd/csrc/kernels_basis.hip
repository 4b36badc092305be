// Per-iteration transforms of the basis and the gradient fold, on the
// row-interleaved internal layouts:
//   W, K : [c][row][x][j]   the r coefficients of one (coil, k-space row, x)
//                           are contiguous (row = sampled line u for 1D
//                           Cartesian masks, ky for general masks);
//   yu   : per sampled line, [c][p][x] over the line's samples p (1D Cartesian);
//   G    : [p][j]            the gradient, pixel-major.
// A workgroup transforms all r basis columns of a tile of txx image columns
// together: LDS holds N x (txx*r) points, loads and stores are whole
// contiguous rows.
//
//   forward  W_{c,j} = F_y(s_c o u_j) on the sampled rows (then F_x for
//            general masks),
//   fold     K_c(row,x,:) = W_c(row,x,:) S_row - sum_{samples on row} y conj(b_k)
//            (the frames' scatter-sum moved before the inverse transform),
//   adjoint  G(:, j) = sum_c conj(s_c) o F_y^H K_{c,j} (after F_x^H for general
//            masks), summed over a coil group per workgroup.
#include "kernels_core.hpp"

namespace ag {

// ---------------------------------------------------------------------------
// forward: grid (nx/txx, coil groups); the U tile stays in registers while
// the workgroup loops over its coils.
// ---------------------------------------------------------------------------
template <int N, int CT>
__global__ __launch_bounds__(AG_NT) void k_basis_fwd(BasisArgs a) {
  __shared__ float2 s[N * CT];
  constexpr int IT = (N * CT + AG_NT - 1) / AG_NT;
  const int tid = threadIdx.x;
  const int txx = a.txx, r = a.r, ctr = txx * r;
  const int x0 = blockIdx.x * txx;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  float2 uv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * AG_NT;
    const int y = g / CT, col = g % CT;
    uv[it] = (g < N * CT && col < ctr) ? a.U[((long)y * a.nx + x0) * r + col] : make_float2(0.f, 0.f);
  }
  const int n_rows = a.rows ? *a.n_rows_ptr : N;
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  float2 cv[IT];
  auto fetch = [&](int c) {
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      const int y = g / CT, col = g % CT;
      cv[it] = (g < N * CT && col < ctr) ? coil[(long)y * a.nx + x0 + col / r] : make_float2(0.f, 0.f);
    }
  };
  if (cb < ce) fetch(cb);
  for (int c = cb; c < ce; ++c) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < N * CT) s[g] = cmul(cv[it], uv[it]);
    }
    __syncthreads();
    if (c + 1 < ce) fetch(c + 1);  // in flight during this coil's transform
    fft_lds<N, CT, AG_NT, false>(s, a.tw);
    float2* dst = a.W + (long)c * a.ua * a.nx * r;
    for (int g = tid; g < n_rows * ctr; g += AG_NT) {
      const int u = g / ctr, col = g - u * ctr;
      const int ky = a.rows ? a.rows[u] : u;
      dst[((long)u * a.nx + x0) * r + col] = cscale(s[ky * CT + col], a.scale);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// adjoint + coil combine: grid (nx/txx, coil groups); group g writes its
// partial gradient to G + g*part_stride.
// ---------------------------------------------------------------------------
template <int N, int CT>
__global__ __launch_bounds__(AG_NT) void k_basis_adj(BasisArgs a) {
  __shared__ float2 s[N * CT];
  constexpr int IT = (N * CT + AG_NT - 1) / AG_NT;
  const int tid = threadIdx.x;
  const int txx = a.txx, r = a.r, ctr = txx * r;
  const int x0 = blockIdx.x * txx;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  const int n_rows = a.rows ? *a.n_rows_ptr : N;
  const bool full = (a.rows == nullptr);
  const int total = n_rows * ctr;  // <= N * CT
  // LDS destination of this thread's row items (fixed across coils)
  int dst[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * AG_NT;
    dst[it] = -1;
    if (g < total) {
      const int u = g / ctr, col = g - u * ctr;
      dst[it] = (full ? u : a.rows[u]) * CT + col;
    }
  }
  float2 acc[IT], kv[IT], cv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) acc[it] = make_float2(0.f, 0.f);
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  // coil c's K rows and coil values, into registers
  auto fetch = [&](int c) {
    const float2* src = a.K + (long)c * a.ua * a.nx * r;
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < total) {
        const int u = g / ctr, col = g - u * ctr;
        kv[it] = src[((long)u * a.nx + x0) * r + col];
      }
      const int y = g / CT, col = g % CT;
      cv[it] = (g < N * CT && col < ctr) ? coil[(long)y * a.nx + x0 + col / r] : make_float2(0.f, 0.f);
    }
  };
  if (cb < ce) fetch(cb);
  for (int c = cb; c < ce; ++c) {
    if (!full) {
      for (int g = tid; g < N * CT; g += AG_NT) s[g] = make_float2(0.f, 0.f);
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (dst[it] >= 0) s[dst[it]] = kv[it];
    float2 cc[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) cc[it] = cv[it];
    __syncthreads();
    if (c + 1 < ce) fetch(c + 1);  // in flight during this coil's transform
    fft_lds<N, CT, AG_NT, true>(s, a.tw);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int g = tid + it * AG_NT;
      if (g < N * CT) acc[it] = cadd(acc[it], cjmul(cc[it], s[g]));
    }
    __syncthreads();
  }
  float2* out = a.G + (long)blockIdx.y * a.part_stride;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * AG_NT;
    const int y = g / CT, col = g % CT;
    if (g < N * CT && col < ctr) out[((long)y * a.nx + x0) * r + col] = cscale(acc[it], a.scale);
  }
}

// ---------------------------------------------------------------------------
// general masks: the x half of the 2D transform, in place on W or K, one
// workgroup per (coil, ky) row of nx x r values.
// ---------------------------------------------------------------------------
template <int N, int CT, bool INV>
__global__ __launch_bounds__(AG_NT) void k_basis_rows(BasisArgs a) {
  __shared__ float2 s[N * CT];
  const int tid = threadIdx.x, r = a.r;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  float2* row = (INV ? a.K : a.W) + (long)blockIdx.x * N * r;
  for (int g = tid; g < N * CT; g += AG_NT) {
    const int x = g / CT, j = g % CT;
    s[g] = (j < r) ? row[(long)x * r + j] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<N, CT, AG_NT, INV>(s, a.tw_x);
  for (int g = tid; g < N * CT; g += AG_NT) {
    const int x = g / CT, j = g % CT;
    if (j < r) row[(long)x * r + j] = cscale(s[g], a.scale_x);
  }
}

// ---------------------------------------------------------------------------
// setup: per-line data yu[nc*nx*p0 + (c*np + p)*nx + x] from the hybrid
// frame-major y'[k][c][l][x]; grid (pairs, nc).
// ---------------------------------------------------------------------------
__global__ void k_build_yu(const float2* yh, const int2* pairs, const int32_t* mask, const int32_t* loc_ptr,
                           int n_loc, int width, int nc, int nx, int lmax, float2* yu, const DevState* st) {
  if (st->err) return;
  const int P = blockIdx.x, c = blockIdx.y;
  if (P >= loc_ptr[n_loc]) return;  // grid covers the largest possible pair count
  const int2 kl = pairs[P];
  const int ky = mask[(long)kl.x * width + kl.y];
  const int p0 = loc_ptr[ky], np = loc_ptr[ky + 1] - p0, p = P - p0;
  const float2* src = yh + (((long)kl.x * nc + c) * lmax + kl.y) * nx;
  float2* dst = yu + (long)nc * nx * p0 + ((long)c * np + p) * nx;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) dst[x] = src[x];
}

// ---------------------------------------------------------------------------
// gradient fold, 1D Cartesian: grid (sampled lines, nc).  The (coil, line)
// block of W (nx x r, contiguous) is staged through LDS with coalesced
// loads, every thread forms one x row of K, and the K block leaves through
// LDS again; the samples' data are read along x.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_fold_lines2(FoldArgs a) {
  __shared__ float2 S[RT * RT];
  __shared__ float2 bc[128 * RT];
  __shared__ float2 Wl[AG_NT * (RT + 1)];
  const int u = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  if (u >= a.st->n_units) return;
  const int r = a.r, nx = a.nx;
  const int ky = a.unit_loc[u];
  const int p0 = a.loc_ptr[ky], np = a.loc_ptr[ky + 1] - p0;
  // S_u and conj(b_k) of the line's samples, prepared once per iteration
  for (int e = tid; e < r * r; e += AG_NT) S[(e / r) * RT + (e % r)] = a.S[(long)u * r * r + e];
  for (int e = tid; e < np * r; e += AG_NT) bc[(e / r) * RT + (e % r)] = a.bcp[(long)p0 * r + e];
  const long blk = ((long)c * a.ua + u) * nx * r;
  const float2* Yb = a.yu + (long)a.nc * nx * p0 + (long)c * np * nx;  // [p][x]
  for (int x0 = 0; x0 < nx; x0 += AG_NT) {
    const int nxc = min(AG_NT, nx - x0);
    if (x0 > 0) __syncthreads();
    for (int g = tid; g < nxc * r; g += AG_NT) Wl[(g / r) * (RT + 1) + (g % r)] = a.W[blk + (long)x0 * r + g];
    __syncthreads();
    if (tid < nxc) {
      const int x = x0 + tid;
      float2 w[RT], kk[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) w[i] = (i < r) ? Wl[tid * (RT + 1) + i] : make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < RT; ++i)
          if (i < r) acc = cadd(acc, cmul(w[i], S[i * RT + j]));
        kk[j] = acc;
      }
#pragma unroll 8
      for (int p = 0; p < np; ++p) {
        const float2 yv = Yb[(long)p * nx + x];
#pragma unroll
        for (int j = 0; j < RT; ++j) kk[j] = csub(kk[j], cmul(yv, bc[p * RT + j]));
      }
#pragma unroll
      for (int j = 0; j < RT; ++j)
        if (j < r) Wl[tid * (RT + 1) + j] = kk[j];
    }
    __syncthreads();
    for (int g = tid; g < nxc * r; g += AG_NT) a.K[blk + (long)x0 * r + g] = Wl[(g / r) * (RT + 1) + (g % r)];
  }
}

// per sampled line: S_u = sum_{samples on u} b_k b_k^H and conj(b_k) per sample
__global__ __launch_bounds__(64) void k_line_S(FoldArgs a) {
  const int u = blockIdx.x, tid = threadIdx.x;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  if (u >= a.st->n_units) return;
  const int r = a.r;
  const int ky = a.unit_loc[u];
  const int p0 = a.loc_ptr[ky], np = a.loc_ptr[ky + 1] - p0;
  for (int e = tid; e < np * r; e += 64) {
    const int p = e / r, j = e % r;
    const float2 b = a.B[(long)a.pairs[p0 + p].x * r + j];
    a.bcp[(long)(p0 + p) * r + j] = make_float2(b.x, -b.y);
  }
  for (int e = tid; e < r * r; e += 64) {
    const int i = e / r, j = e % r;
    float2 sacc = make_float2(0.f, 0.f);
    for (int p = 0; p < np; ++p) {
      const float2* b = a.B + (long)a.pairs[p0 + p].x * r;
      sacc = cadd(sacc, cmulj(b[i], b[j]));
    }
    a.S[(long)u * r * r + e] = sacc;
  }
}

// gradient fold, general masks: per location and coil,
//   K_c(loc,:) = sum_{(k,e) at loc} (W_c(loc,:) b_k - y_{k,c}(e)) conj(b_k)
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_fold_index2(FoldArgs a) {
  const int loc = blockIdx.x * AG_NT + threadIdx.x, c = blockIdx.y;
  if (a.st->err || (a.check_halt && a.st->halt)) return;
  if (loc >= a.n) return;
  const int r = a.r;
  const long base = ((long)c * a.n + loc) * r;
  float2 w[RT], kk[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    w[i] = (i < r) ? a.W[base + i] : make_float2(0.f, 0.f);
    kk[i] = make_float2(0.f, 0.f);
  }
  const int p0 = a.loc_ptr[loc], p1 = a.loc_ptr[loc + 1];
  for (int p = p0; p < p1; ++p) {
    const int2 ke = a.pairs[p];
    const float2* b = a.B + (long)ke.x * r;
    float2 bb[RT];
    float2 res = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      bb[i] = (i < r) ? b[i] : make_float2(0.f, 0.f);
      res = cadd(res, cmul(w[i], bb[i]));
    }
    res = csub(res, a.y[((long)ke.x * a.nc + c) * a.m_max + ke.y]);
#pragma unroll
    for (int j = 0; j < RT; ++j) kk[j] = cadd(kk[j], cmulj(res, bb[j]));
  }
#pragma unroll
  for (int j = 0; j < RT; ++j)
    if (j < r) a.K[base + j] = kk[j];
}

// column-major (the C ABI's n x r layout) -> pixel-major r columns
__global__ void k_to_pixmajor(const float2* src, int r, long n, float2* dst) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long step = (long)gridDim.x * blockDim.x;
  for (; i < n * r; i += step) {
    const long p = i / r, j = i % r;
    dst[i] = src[j * n + p];
  }
}

// pixel-major r columns -> column-major (the C ABI's n x r layout)
__global__ void k_to_colmajor(const float2* src, int r, long n, float2* dst) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long step = (long)gridDim.x * blockDim.x;
  for (; i < n * r; i += step) {
    const long p = i % n, j = i / n;
    dst[i] = src[p * r + j];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int basis_ct(int N) { return N >= 256 ? 16 : (N >= 128 ? 32 : 64); }

int basis_txx(int N, int nx, int r) {
  const int ct = basis_ct(N);
  int t = 1;
  while (2 * t * r <= ct && 2 * t <= nx) t *= 2;
  return t;
}

template <int N>
static void launch_basis_n(int which, const BasisArgs& a, int grid_x, int grid_y, hipStream_t s) {
  constexpr int CT = N >= 256 ? 16 : (N >= 128 ? 32 : 64);
  const dim3 g(grid_x, grid_y);
  if (which == 0) hipLaunchKernelGGL((k_basis_fwd<N, CT>), g, dim3(AG_NT), 0, s, a);
  else if (which == 1) hipLaunchKernelGGL((k_basis_adj<N, CT>), g, dim3(AG_NT), 0, s, a);
  else if (which == 2) hipLaunchKernelGGL((k_basis_rows<N, CT, false>), g, dim3(AG_NT), 0, s, a);
  else hipLaunchKernelGGL((k_basis_rows<N, CT, true>), g, dim3(AG_NT), 0, s, a);
}

hipError_t launch_basis(int which, int N, const BasisArgs& a, int grid_x, int grid_y, hipStream_t s) {
  switch (N) {
    case 8: launch_basis_n<8>(which, a, grid_x, grid_y, s); break;
    case 16: launch_basis_n<16>(which, a, grid_x, grid_y, s); break;
    case 32: launch_basis_n<32>(which, a, grid_x, grid_y, s); break;
    case 64: launch_basis_n<64>(which, a, grid_x, grid_y, s); break;
    case 128: launch_basis_n<128>(which, a, grid_x, grid_y, s); break;
    case 256: launch_basis_n<256>(which, a, grid_x, grid_y, s); break;
    case 512: launch_basis_n<512>(which, a, grid_x, grid_y, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fold2(const FoldArgs& a, bool lines, int grid_x, int grid_y, hipStream_t s) {
  const dim3 g(grid_x, grid_y);
  if (lines) {
    hipLaunchKernelGGL(k_line_S, dim3(grid_x), dim3(64), 0, s, a);
    if (a.r <= 4) hipLaunchKernelGGL(k_fold_lines2<4>, g, dim3(AG_NT), 0, s, a);
    else if (a.r <= 8) hipLaunchKernelGGL(k_fold_lines2<8>, g, dim3(AG_NT), 0, s, a);
    else hipLaunchKernelGGL(k_fold_lines2<16>, g, dim3(AG_NT), 0, s, a);
  } else {
    if (a.r <= 4) hipLaunchKernelGGL(k_fold_index2<4>, g, dim3(AG_NT), 0, s, a);
    else if (a.r <= 8) hipLaunchKernelGGL(k_fold_index2<8>, g, dim3(AG_NT), 0, s, a);
    else hipLaunchKernelGGL(k_fold_index2<16>, g, dim3(AG_NT), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace ag
