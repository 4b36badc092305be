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
#include "mma.hpp"

namespace ag {

template <int N>
__device__ __forceinline__ constexpr bool PL_ONE() { return FftPlan<N>::P == 1; }

// ---------------------------------------------------------------------------
// forward: grid (nx/txx, coil groups).  The U tile and the coil values feed
// the transform's first pass straight from registers and the last pass
// stores straight to W, so per coil only the middle of the transform goes
// through LDS; the next coil's values are loaded during the transform.
// ---------------------------------------------------------------------------
template <int N, int CT>
__global__ __launch_bounds__(AG_NT) void k_basis_fwd(BasisArgs a) {
  using GM = FftGeom<N, CT, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  __shared__ float2 s[FftPlan<N>::P > 1 ? N * CT : 1];
  __shared__ float2 s_tw[N];
  __shared__ int s_ro[N];  // k-space row -> offset of its W row within a coil, -1 if not kept
  const int tid = threadIdx.x;
  const int txx = a.txx, r = a.r, ctr = txx * r;
  const int x0 = blockIdx.x * txx;
  // the U tile and the first coil's values are requested first, then the
  // tables (both loads before either store), then the state: one round trip
  // (loads from clamped, valid addresses, not under a branch; elements out
  // of the tile are zeroed where U and the coil values are multiplied)
  bool okg[IT0];
  float2 uv[IT0][R0];
#pragma unroll
  for (int it = 0; it < IT0; ++it) {
    const int g0 = tid + it * AG_NT;
    okg[it] = GM::in_ok(g0) && (g0 % CT) < ctr;
    const int g = okg[it] ? g0 : 0, col = g % CT;
#pragma unroll
    for (int q = 0; q < R0; ++q) uv[it][q] = a.U[((long)GM::in_row(g, q) * a.nx + x0) * r + col];
  }
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  float2 cv[IT0][R0];
  auto fetch = [&](int c) {
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
      const int g = okg[it] ? tid + it * AG_NT : 0, col = g % CT;
      const float2* cp = coil + (long)blockIdx.x * N * txx + (g / CT) * txx + col / r;  // [x/txx][y][x%txx]
#pragma unroll
      for (int q = 0; q < R0; ++q) cv[it][q] = cp[q * (N / R0) * txx];
    }
  };
  if (cb < ce) fetch(cb);
  for (int e = tid; e < N; e += AG_NT) {
    const float2 t = a.tw[e];
    const int u = a.row_unit ? a.row_unit[e] : e;
    s_tw[e] = t;
    s_ro[e] = u >= 0 ? u * a.nx * r : -1;
  }
  // the state is read once the first loads are in flight (their addresses are valid either way)
  if (halted(a.st, a.check_halt)) return;
  __syncthreads();
  for (int c = cb; c < ce; ++c) {
    float2 v0[IT0][R0], vo[ITL][RL];
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int q = 0; q < R0; ++q) v0[it][q] = okg[it] ? cmul(cv[it][q], uv[it][q]) : make_float2(0.f, 0.f);
    if (c + 1 < ce) fetch(c + 1);
    fft_regs<N, CT, AG_NT, false>(v0, vo, s, s_tw);
    float2* dst = a.W + (long)c * a.ua * a.nx * r + x0 * r;
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int g = tid + it * AG_NT, col = g % CT;
      if (GM::out_ok(g) && col < ctr) {
#pragma unroll
        for (int q = 0; q < RL; ++q) {
          const int ro = s_ro[GM::out_row(g, q)];
          if (ro >= 0) dst[ro + col] = cscale(vo[it][q], a.scale);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint + coil combine: grid (nx/txx, coil groups); group g writes its
// partial gradient to G + g*part_stride.  K rows feed the first pass from
// registers (zero on rows that are not sampled), the coil-weighted sum is
// taken on the last pass's registers.
// ---------------------------------------------------------------------------
template <int N, int CT>
__global__ __launch_bounds__(AG_NT) void k_basis_adj(BasisArgs a) {
  using GM = FftGeom<N, CT, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  __shared__ float2 s[FftPlan<N>::P > 1 ? N * CT : 1];
  __shared__ float2 s_tw[N];
  __shared__ int s_ro[N];  // k-space row -> offset of its K row within a coil, -1 for a zero row
  const int tid = threadIdx.x;
  const int txx = a.txx, r = a.r, ctr = txx * r;
  const int x0 = blockIdx.x * txx;
  for (int e = tid; e < N; e += AG_NT) {  // both loads before either store: one round trip
    const float2 w = a.tw[e];
    const int u = a.row_unit ? a.row_unit[e] : e;
    s_tw[e] = make_float2(w.x, -w.y);
    s_ro[e] = u >= 0 ? u * a.nx * r : -1;
  }
  __syncthreads();
  float2 acc[ITL][RL];
#pragma unroll
  for (int it = 0; it < ITL; ++it)
#pragma unroll
    for (int q = 0; q < RL; ++q) acc[it][q] = make_float2(0.f, 0.f);
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  float2 kv[IT0][R0];
  auto fetch = [&](int c) {
    const float2* src = a.K + (long)c * a.ua * a.nx * r + x0 * r;
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
      const int g = tid + it * AG_NT, col = g % CT;
      const bool ok = GM::in_ok(g) && col < ctr;
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const int ro = ok ? s_ro[GM::in_row(g, q)] : -1;
        kv[it][q] = ro >= 0 ? src[ro + col] : make_float2(0.f, 0.f);
      }
    }
  };
  if (cb < ce) fetch(cb);
  // the state is read once the first loads are in flight (their addresses are valid either way)
  if (halted(a.st, a.check_halt)) return;
  for (int c = cb; c < ce; ++c) {
    float2 v0[IT0][R0], vo[ITL][RL];
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int q = 0; q < R0; ++q) v0[it][q] = kv[it][q];
    if (c + 1 < ce) fetch(c + 1);
    // the forward table conjugated in LDS gives the inverse twiddles
    fft_regs<N, CT, AG_NT, true>(v0, vo, s, s_tw);
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int g = tid + it * AG_NT, col = g % CT;
      if (GM::out_ok(g) && col < ctr) {
        const float2* cp = coil + (long)blockIdx.x * N * txx + (g / CT) * (PL_ONE<N>() ? RL : 1) * txx + col / r;
#pragma unroll
        for (int q = 0; q < RL; ++q) {
          const float2 cw = cp[(PL_ONE<N>() ? q : q * (N / RL)) * txx];
          acc[it][q] = cjfma(acc[it][q], cw, vo[it][q]);
        }
      }
    }
  }
  float2* out = a.G + (long)blockIdx.y * a.part_stride;
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int g = tid + it * AG_NT, col = g % CT;
    if (GM::out_ok(g) && col < ctr) {
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        const int y = GM::out_row(g, q);
        out[((long)y * a.nx + x0) * r + col] = cscale(acc[it][q], a.scale);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint + coil combine over every coil + the QR step's Gram partial, one
// image column x per workgroup (r <= 16, one block of the QR Gram per column):
// grid nx (consecutive columns on one XCD, which then share the cache lines
// of K, G and U), 512 threads in two groups of 256.  A transform tile holds
// ncp = CT / r coils' r columns of K(:, x, :); the two groups transform
// alternate coil passes into their own accumulators.  Then
//   G(y, x, :) = scale * sum_c conj(s_c(y, x)) F_y^H K_c(:, x, :)
// (the groups' and coil slots' terms added in a fixed order) is stored, and
// the real-embedded Gram [Re U, Re G, Im U, Im G]^T [...] over the column's
// N pixels is formed on the matrix cores; its complex upper triangle (tri
// order over the 2r columns [U G], FP32) goes to qpart[blockIdx.x], the
// block partial that the QR step sums.
// ---------------------------------------------------------------------------
template <int N, int CT, int TRM>
__global__ __launch_bounds__(512) void k_adj_qr(BasisArgs a) {
  using GM = FftGeom<N, CT, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  // the real embedding of [U G] has 4r <= 16 TRM columns: TRM row tiles, NTL upper tiles
  constexpr int NTL = TRM * (TRM + 1) / 2, EC = 16 * TRM;
  // row pitch of the embedding: a step's 4 rows in disjoint bank quarters
  constexpr int LDX = (EC % 64 == 0 || EC % 64 == 32) ? EC + 16 : EC;
  constexpr int UE = (N * 4 * TRM + 511) / 512;  // U entries per thread (r <= 4 TRM)
  constexpr int CMAX = 3072;  // coil values of the column staged in LDS when nc N fits
  // one LDS block: the two transform tiles, then the embedding X (the staged
  // coil values share its space: they are done with before X is formed);
  // after the matrix-core loop both serve as the scratch of the reduction
  constexpr int S_BYTES = 2 * N * CT * 8;
  constexpr int XS_BYTES = (N * LDX * 4 > CMAX * 8) ? N * LDX * 4 : CMAX * 8;
  static_assert(8 * NTL * 256 * 4 <= S_BYTES + XS_BYTES, "reduction scratch");
  __shared__ __attribute__((aligned(16))) char lds_blk[S_BYTES + XS_BYTES];
  float2 (*s)[N * CT] = reinterpret_cast<float2 (*)[N * CT]>(lds_blk);
  float* const X = reinterpret_cast<float*>(lds_blk + S_BYTES);
  float2* const s_cw = reinterpret_cast<float2*>(lds_blk + S_BYTES);
  __shared__ float red[NTL * 256];
  __shared__ float2 s_tw[N];
  __shared__ int s_ro[N];  // k-space row -> offset of its K row within a coil, -1 for a zero row
  const int tid = threadIdx.x, grp = tid >> 8, lt = tid & 255;
  const int r = a.r, nx = a.nx, ncp = CT / r, nct = ncp * r, txx = a.txx;
  const bool cw_lds = a.nc * N <= CMAX;
  const int b = blockIdx.x;
  const int x = (nx % 8 == 0) ? (b % 8) * (nx / 8) + b / 8 : b;
  // the column's basis rows U(y, x, :) for the Gram (pixel-major U), requested first
  float2 uv[UE];
#pragma unroll
  for (int i = 0; i < UE; ++i) {
    const int e = min(tid + 512 * i, N * r - 1), y = e / r, j = e - y * r;
    uv[i] = a.U[((long)y * nx + x) * r + j];
  }
  for (int e = tid; e < N; e += 512) {
    const float2 w = a.tw[e];
    const int u = a.row_unit ? a.row_unit[e] : e;
    s_tw[e] = make_float2(w.x, -w.y);
    s_ro[e] = u >= 0 ? u * nx * r : -1;
  }
  // the column's coil values s_c(y, x) for every coil: the combine then reads LDS
  if (cw_lds)
    for (int e = tid; e < a.nc * N; e += 512) {
      const int c = e / N, y = e - c * N;
      s_cw[e] = a.coils[(long)c * a.n + (long)(x / txx) * N * txx + (long)y * txx + (x % txx)];
    }
  __syncthreads();
  const int npass = (a.nc + ncp - 1) / ncp, nround = (npass + 1) / 2;
  float2 acc[ITL][RL];
#pragma unroll
  for (int it = 0; it < ITL; ++it)
#pragma unroll
    for (int q = 0; q < RL; ++q) acc[it][q] = make_float2(0.f, 0.f);
  float2 kv[IT0][R0];
  auto fetch = [&](int pass) {  // a pass past the last coil gives zeros
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
      const int g = lt + it * AG_NT, col = g % CT, cs = col / r, j = col - cs * r, c = pass * ncp + cs;
      const bool ok = GM::in_ok(g) && col < nct && c < a.nc;
      const float2* src = a.K + (long)(ok ? c : 0) * a.ua * nx * r + x * r + j;
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const int ro = ok ? s_ro[GM::in_row(g, q)] : -1;
        kv[it][q] = ro >= 0 ? src[ro] : make_float2(0.f, 0.f);
      }
    }
  };
  fetch(grp);
  // the state is read once the first loads are in flight; the test is the
  // same in every thread
  if (halted(a.st, a.check_halt)) return;
  for (int rd = 0; rd < nround; ++rd) {  // both groups run every round (and reach every barrier)
    const int pass = grp + 2 * rd;
    float2 v0[IT0][R0], vo[ITL][RL];
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int q = 0; q < R0; ++q) v0[it][q] = kv[it][q];
    if (rd + 1 < nround) fetch(pass + 2);
    fft_regs<N, CT, AG_NT, true>(v0, vo, s[grp], s_tw);
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int g = lt + it * AG_NT, col = g % CT, cs = col / r, c = pass * ncp + cs;
      if (GM::out_ok(g) && col < nct && c < a.nc) {
        if (cw_lds) {
#pragma unroll
          for (int q = 0; q < RL; ++q) acc[it][q] = cjfma(acc[it][q], s_cw[c * N + GM::out_row(g, q)], vo[it][q]);
        } else {
          const float2* cp = a.coils + (long)c * a.n + (long)(x / txx) * N * txx + (x % txx);
#pragma unroll
          for (int q = 0; q < RL; ++q)
            acc[it][q] = cjfma(acc[it][q], cp[(long)GM::out_row(g, q) * txx], vo[it][q]);
        }
      }
    }
  }
  // each group's terms to its tile (free after the last transform's barrier)
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int g = lt + it * AG_NT;
    if (GM::out_ok(g)) {
#pragma unroll
      for (int q = 0; q < RL; ++q) s[grp][GM::out_row(g, q) * CT + g % CT] = acc[it][q];
    }
  }
  __syncthreads();
  // the column's gradient, stored and embedded with U; embedding columns
  // from 4r on stay zero
  const int m = 2 * r;
  for (int e = tid; e < N * EC; e += 512) {
    const int y = e / EC, k = e % EC;
    if (k >= 2 * m) X[y * LDX + k] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < UE; ++i) {
    const int e = tid + 512 * i;
    if (e < N * r) {
      const int y = e / r, j = e - y * r;
      float2 v = make_float2(0.f, 0.f);
      for (int h = 0; h < 2; ++h)
        for (int cs = 0; cs < ncp; ++cs) v = cadd(v, s[h][y * CT + cs * r + j]);
      v = cscale(v, a.scale);
      a.G[((long)y * nx + x) * r + j] = v;
      X[y * LDX + j] = uv[i].x;
      X[y * LDX + m + j] = uv[i].y;
      X[y * LDX + r + j] = v.x;
      X[y * LDX + m + r + j] = v.y;
    }
  }
  __syncthreads();
  // the Gram on the matrix cores: wave w takes rows [w N/8, (w+1) N/8), 4 per step
  using M = Mma<float>;
  const int wave = tid >> 6, lane = tid & 63, mc = lane & 15, kk = lane >> 4;
  M::V gacc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) gacc[t] = M::zero();
#pragma unroll
  for (int st = 0; st < N / 32; ++st) {
    const float* xr = X + ((N / 8) * wave + 4 * st + kk) * LDX + mc;
    float xv[TRM];
#pragma unroll
    for (int t = 0; t < TRM; ++t) xv[t] = xr[16 * t];
#pragma unroll
    for (int i = 0; i < TRM; ++i)
#pragma unroll
      for (int j = i; j < TRM; ++j) {
        const int ti = i * TRM - i * (i - 1) / 2 + (j - i);
        gacc[ti] = M::mma(xv[i], xv[j], gacc[ti]);
      }
  }
  // once every wave's matrix-core reads of X are done, the whole block is
  // the scratch for the sum over the waves
  __syncthreads();
  tiles_reduce_par<float, 8, NTL>(red, reinterpret_cast<float*>(lds_blk), gacc, wave, lane);
  auto C = [&](int i, int j) -> float {
    if (i > j) {
      const int t = i;
      i = j;
      j = t;
    }
    const int a_ = i / 16, b_ = j / 16;
    return red[(a_ * TRM - a_ * (a_ - 1) / 2 + (b_ - a_)) * 256 + (i % 16) * 16 + (j % 16)];
  };
  const int nout = m * (m + 1) / 2;
  float2* qp = a.qpart + (long)b * nout;
  for (int o = tid; o < nout; o += 512) {
    int i, j;
    tri_index(o, m, i, j);
    qp[o] = make_float2(C(i, j) + C(m + i, m + j), C(i, m + j) - C(m + i, j));
  }
}

// ---------------------------------------------------------------------------
// general masks: the x half of the 2D transform, in place on W or K.  One
// workgroup per a.txx consecutive (coil, ky) rows of nx x r values, the
// rows side by side as the transform's columns (col = row * r + j); the
// first pass is fed from registers and the last one stays there.
// ---------------------------------------------------------------------------
template <int N, int CT, bool INV>
__global__ __launch_bounds__(AG_NT) void k_basis_rows(BasisArgs a) {
  using GM = FftGeom<N, CT, AG_NT>;
  constexpr int IT0 = GM::IT0, R0 = GM::R0, ITL = GM::ITL, RL = GM::RL;
  __shared__ float2 s[FftPlan<N>::P > 1 ? N * CT : 1];
  __shared__ float2 s_tw[N];
  const int tid = threadIdx.x, r = a.r;
  const int tyy = a.txx, ctr = tyy * r;
  const long nrows = (long)a.nc * a.ua;
  const long row0 = (long)blockIdx.x * tyy;
  float2* const base = (INV ? a.K : a.W) + row0 * N * r;
  // loads from clamped, valid addresses (column 0 of the first row), zeroed
  // outside the tile after the load
  float2 v0[IT0][R0];
  bool okg[IT0];
#pragma unroll
  for (int it = 0; it < IT0; ++it) {
    const int g0 = tid + it * AG_NT, col0 = g0 % CT;
    okg[it] = GM::in_ok(g0) && col0 < ctr && row0 + col0 / r < nrows;
    const int g = okg[it] ? g0 : 0, col = g % CT, yy = col / r, j = col - yy * r;
#pragma unroll
    for (int q = 0; q < R0; ++q) v0[it][q] = base[((long)yy * N + GM::in_row(g, q)) * r + j];
  }
  for (int e = tid; e < N; e += AG_NT) {
    const float2 t = a.tw_x[e];
    s_tw[e] = INV ? make_float2(t.x, -t.y) : t;  // the inverse takes the conjugated table
  }
  if (halted(a.st, a.check_halt)) return;
#pragma unroll
  for (int it = 0; it < IT0; ++it)
#pragma unroll
    for (int q = 0; q < R0; ++q)
      if (!okg[it]) v0[it][q] = make_float2(0.f, 0.f);
  __syncthreads();
  float2 vo[ITL][RL];
  fft_regs<N, CT, AG_NT, INV>(v0, vo, s, s_tw);
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int g = tid + it * AG_NT, col = g % CT, yy = col / r, j = col - yy * r;
    if (GM::out_ok(g) && col < ctr && row0 + yy < nrows) {
#pragma unroll
      for (int q = 0; q < RL; ++q) base[((long)yy * N + GM::out_row(g, q)) * r + j] = cscale(vo[it][q], a.scale_x);
    }
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
// gradient fold, 1D Cartesian: per sampled line u and coil c,
//   K_c[u][x][:] = sum_{p in u} (W_c[u][x][:] . b_p - y_p(c, x)) conj(b_p)^T
// over the line's (frame, line) pairs p: the residual of every sample times
// conj(b) of its frame.  One workgroup per (line, coil); thread = readout
// position x, holding its row of r values in registers (rows of even r move
// as float4).  conj(b_p) of the line's pairs are staged in LDS.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_fold_lines2(FoldArgs a) {
  __shared__ float2 bc[128 * RT];  // conj(b_p) of the line's pairs (at most q <= 128)
  // grid (coils, rows): the lines with the most pairs first; the record of
  // a row position past the sampled lines names an unsampled row below n_loc,
  // so u is in range before it is checked
  const int4 lrec = a.line_order[blockIdx.y];
  const int u = lrec.x, c = blockIdx.x, tid = threadIdx.x;
  const int r = a.r, nx = a.nx;
  const bool vec = (r & 1) == 0;
  float2 w[RT];
  auto load_w = [&](int x0) {
    const float2* src = a.W + (((long)c * a.ua + u) * nx + min(x0 + tid, nx - 1)) * r;
    if (vec) {
#pragma unroll
      for (int i = 0; i < RT; i += 2) {
        const float4 v = (i < r) ? *reinterpret_cast<const float4*>(src + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        w[i] = make_float2(v.x, v.y);
        w[i + 1] = make_float2(v.z, v.w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < RT; ++i) w[i] = (i < r) ? src[i] : make_float2(0.f, 0.f);
    }
  };
  // the first chunk's W rows are requested before the state is read (every
  // address is valid either way), so that the latencies overlap; the span is
  // used only once the line is known to be sampled
  load_w(0);
  const int nu_ = a.st->n_units;  // requested with the stop test's loads
  if (halted(a.st, a.check_halt) || u >= nu_) return;
  const int p0 = lrec.y, np = lrec.z;
  const float2* Yc = a.yu + (long)a.nc * nx * p0 + (long)c * np * nx;  // this line and coil, [p][x]
  float2 ya[8], yb[8];
  auto load_y = [&](int x0, int pb, float2 (&yv)[8]) {
    const int x = min(x0 + tid, nx - 1);
#pragma unroll
    for (int t = 0; t < 8; ++t) yv[t] = (pb + t < np) ? Yc[(long)(pb + t) * nx + x] : make_float2(0.f, 0.f);
  };
  load_y(0, 0, ya);
  // padding entries (j >= r) are zero, so whole RT-wide rows can be used
  for (int e = tid; e < np * RT; e += AG_NT) {
    const int p = e / RT, j = e - p * RT;
    bc[e] = (j < r) ? a.bcp[(long)(p0 + p) * r + j] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // one pair: kk += (w . b_p - y) conj(b_p)
  auto pair = [&](int p, float2 yv, float2 (&kk)[RT]) {
    const float2* bp = bc + p * RT;
    float2 res = make_float2(-yv.x, -yv.y);
#pragma unroll
    for (int i = 0; i < RT; ++i) res = cfmaj(res, w[i], bp[i]);
#pragma unroll
    for (int j = 0; j < RT; ++j) kk[j] = cfma(kk[j], res, bp[j]);
  };
  for (int x0 = 0; x0 < nx; x0 += AG_NT) {
    if (x0 > 0) {
      load_w(x0);
      load_y(x0, 0, ya);
    }
    float2 kk[RT];
#pragma unroll
    for (int j = 0; j < RT; ++j) kk[j] = make_float2(0.f, 0.f);
    // data batches of 8, the next batch in flight while this one is used
    for (int pb = 0; pb < np; pb += 16) {
      if (pb + 8 < np) load_y(x0, pb + 8, yb);
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (pb + t < np) pair(pb + t, ya[t], kk);
      if (pb + 8 >= np) break;
      if (pb + 16 < np) load_y(x0, pb + 16, ya);
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (pb + 8 + t < np) pair(pb + 8 + t, yb[t], kk);
    }
    if (x0 + tid < nx) {
      float2* dst = a.K + (((long)c * a.ua + u) * nx + x0 + tid) * r;
      if (vec) {
#pragma unroll
        for (int j = 0; j < RT; j += 2)
          if (j < r) *reinterpret_cast<float4*>(dst + j) = make_float4(kk[j].x, kk[j].y, kk[j + 1].x, kk[j + 1].y);
      } else {
#pragma unroll
        for (int j = 0; j < RT; ++j)
          if (j < r) dst[j] = kk[j];
      }
    }
  }
}

// gradient fold, 1D Cartesian, on the matrix cores: per (line u, coil c)
//   K(x, :) = sum_{p in u} (W(x, :) . b_p - y_p(x)) conj(b_p)^T
//           = [W(x, :) | y_1(x) .. y_np(x)] . [S_u ; -conj(b_1)^T ; ...]
// with S_u = sum_p b_p b_p^H: one complex contraction per row x of length
// r + np, run as a real one (v_mfma_f32_16x16x4f32) over the contraction
// index kappa = [Re W_0..RT-1, Im W_0..RT-1, (Re y_p, Im y_p) for every pair]
// and the 2 RT output columns [Re K_0..RT-1, Im K_0..RT-1]:
//   Re W_i  -> [ Re S_ij |  Im S_ij ]      Im W_i -> [ -Im S_ij | Re S_ij ]
//   Re y_p  -> [ -Re b_pj |  Im b_pj ]     Im y_p -> [ -Im b_pj | -Re b_pj ]
// The B operand (kappa x 2 RT) is built in LDS from the pairs' b; each wave
// takes 16-row tiles of x, its A operand straight from W and the line data
// (lane l: row l % 16, contraction slot l / 16), and writes each tile's 16
// contiguous K rows through LDS.  Accumulation order is fixed.
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_fold_lines_mma(FoldArgs a) {
  typedef float fv4 __attribute__((ext_vector_type(4)));
  constexpr int NCOL = 2 * RT, NCT = NCOL / 16;
  constexpr int TW = 4;                   // 16-row tiles per wave, worked together (nx <= 256)
  constexpr int YB = 4;                   // contraction steps of line data loaded per batch
  // dynamic LDS sized by the launch for at most a.max_pairs pairs per line:
  // b_p (not conjugated, zero for j >= r), then the B operand
  extern __shared__ float2 fold_lds[];
  float2* bb = fold_lds;
  float* Bm = reinterpret_cast<float*>(fold_lds + a.max_pairs * RT);
  __shared__ float spart[4][RT * RT * 2];  // S_u partial sums over four slices of the pairs
  constexpr int OP = NCOL + 4;            // output-tile row pitch: the 4 row groups of a store fall in distinct banks
  __shared__ float ot[4][16 * OP];        // one output tile per wave
  const int4 lrec = a.line_order[blockIdx.y];
  const int u = lrec.x, c = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, row = lane & 15, kq = lane >> 4;
  const int r = a.r, nx = a.nx;
  const int ntile = nx / 16;
  const int p0 = lrec.y, np = lrec.z;
  // this wave's W rows, requested first (valid, clamped addresses; the line
  // is checked once they are in flight): slot kq takes W(x, 4 h + kq)
  const float2* Wl = a.W + ((long)c * a.ua + u) * nx * r;
  float2 wv[TW][RT / 4];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int t = min(wave + 4 * tt, ntile - 1);
    const float2* wr = Wl + (t * 16 + row) * r;
#pragma unroll
    for (int h = 0; h < RT / 4; ++h) wv[tt][h] = wr[min(4 * h + kq, r - 1)];
  }
  const int nu_ = a.st->n_units;
  if (halted(a.st, a.check_halt) || u >= nu_) return;
#pragma unroll
  for (int tt = 0; tt < TW; ++tt)
#pragma unroll
    for (int h = 0; h < RT / 4; ++h)
      if (4 * h + kq >= r) wv[tt][h] = make_float2(0.f, 0.f);
  const float2* Yc = a.yu + (long)a.nc * nx * p0 + (long)c * np * nx;  // this line and coil, [p][x]
  const int kap = (2 * RT + 2 * np + 3) & ~3;  // contraction length, padded to the MFMA's 4
  const int nps = (kap - 2 * RT) >> 2;         // steps over the line data: pairs 2s, 2s + 1
  // the first batch of line data: slot kq of step s takes pair 2 s + kq / 2
  int toff[TW];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) toff[tt] = min(wave + 4 * tt, ntile - 1) * 16 + row;
  // each slot needs one component: Re for even kq, Im for odd (a per-lane
  // choice between the two halves of a loaded float2 would become a
  // runtime-indexed private array)
  const float* Yf = reinterpret_cast<const float*>(Yc) + (kq & 1);
  float yv[YB][TW];
#pragma unroll
  for (int h = 0; h < YB; ++h) {
    const int p = min(2 * h + (kq >> 1), np - 1);
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) yv[h][tt] = Yf[2 * (p * nx + toff[tt])];
  }
  __builtin_amdgcn_sched_barrier(0);  // in flight during the B operand's construction
  for (int e = tid; e < np * RT; e += AG_NT) {
    const int p = e / RT, j = e - p * RT;
    const float2 v = (j < r) ? a.bcp[(long)(p0 + p) * r + j] : make_float2(0.f, 0.f);
    bb[e] = make_float2(v.x, -v.y);
  }
  __syncthreads();
  // S_u = sum_p b_p b_p^H: entry (i, j) over four slices of the pairs
  {
    const int sl = tid / (AG_NT / 4), e0 = tid % (AG_NT / 4);
    for (int e = e0; e < RT * RT; e += AG_NT / 4) {
      const int i = e / RT, j = e - i * RT;
      float sr = 0.f, si = 0.f;
      for (int p = sl; p < np; p += 4) {
        const float2 bi = bb[p * RT + i], bj = bb[p * RT + j];
        sr += bi.x * bj.x + bi.y * bj.y;  // b_i conj(b_j)
        si += bi.y * bj.x - bi.x * bj.y;
      }
      spart[sl][2 * e] = sr;
      spart[sl][2 * e + 1] = si;
    }
  }
  // the line data's rows of B
  for (int e = tid; e < (kap - 2 * RT) * RT; e += AG_NT) {
    const int kk = e / RT, j = e - kk * RT, p = kk >> 1;
    const float2 b = (p < np) ? bb[p * RT + j] : make_float2(0.f, 0.f);
    float* br = Bm + (2 * RT + kk) * NCOL;
    if ((kk & 1) == 0) {
      br[j] = -b.x;
      br[RT + j] = b.y;
    } else {
      br[j] = -b.y;
      br[RT + j] = -b.x;
    }
  }
  __syncthreads();
  for (int e = tid; e < RT * RT; e += AG_NT) {
    const int i = e / RT, j = e - i * RT;
    const float sr = (spart[0][2 * e] + spart[1][2 * e]) + (spart[2][2 * e] + spart[3][2 * e]);
    const float si = (spart[0][2 * e + 1] + spart[1][2 * e + 1]) + (spart[2][2 * e + 1] + spart[3][2 * e + 1]);
    Bm[i * NCOL + j] = sr;
    Bm[i * NCOL + RT + j] = si;
    Bm[(RT + i) * NCOL + j] = -si;
    Bm[(RT + i) * NCOL + RT + j] = sr;
  }
  __syncthreads();
  fv4 acc[TW][NCT];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[tt][ct] = fv4{0.f, 0.f, 0.f, 0.f};
  // W part: Re W in the first RT / 4 steps, Im W in the next RT / 4
#pragma unroll
  for (int h = 0; h < RT / 4; ++h)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const float bre = Bm[(4 * h + kq) * NCOL + ct * 16 + row];
      const float bim = Bm[(RT + 4 * h + kq) * NCOL + ct * 16 + row];
#pragma unroll
      for (int tt = 0; tt < TW; ++tt) {
        acc[tt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[tt][h].x, bre, acc[tt][ct], 0, 0, 0);
        acc[tt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[tt][h].y, bim, acc[tt][ct], 0, 0, 0);
      }
    }
  // line-data part: slot kq of step s takes pair 2 s + kq/2, Re (kq even) or
  // Im; a batch's loads are issued together (the first batch with the W rows)
  for (int s0 = 0; s0 < nps; s0 += YB) {
    if (s0 > 0) {
#pragma unroll
      for (int h = 0; h < YB; ++h) {
        const int p = min(2 * (s0 + h) + (kq >> 1), np - 1);
#pragma unroll
        for (int tt = 0; tt < TW; ++tt) yv[h][tt] = Yf[2 * (p * nx + toff[tt])];
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // the batch's loads all issue before the first use
#pragma unroll
    for (int h = 0; h < YB; ++h) {
      if (s0 + h < nps) {
        const int kk = 2 * RT + 4 * (s0 + h) + kq;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const float bv = Bm[kk * NCOL + ct * 16 + row];
#pragma unroll
          for (int tt = 0; tt < TW; ++tt) {
            acc[tt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[h][tt], bv, acc[tt][ct], 0, 0, 0);
          }
        }
      }
    }
  }
  // D[4 kq + v][row] of column tile ct -> out[x][n]; then the tile's 16
  // contiguous rows of r complex values
  float2* Kl = a.K + ((long)c * a.ua + u) * nx * r;
  float* out = ot[wave];
  const bool full = (r == RT);
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int t = wave + 4 * tt;
    if (t < ntile) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(4 * kq + v) * OP + ct * 16 + row] = acc[tt][ct][v];
      // the tile is read back by other lanes of this wave: a wave's LDS
      // operations execute in order, so only the compiler must keep them so
      // (a memory fence here would also wait for the wave's global stores)
      __builtin_amdgcn_wave_barrier();
      float2* dst = Kl + (long)t * 16 * r;
      if (full) {  // 16 RT contiguous values, RT / 4 per lane
#pragma unroll
        for (int e0 = 0; e0 < 16 * RT; e0 += 64) {
          const int e = e0 + lane, xr = e / RT, j = e % RT;
          dst[e] = make_float2(out[xr * OP + j], out[xr * OP + RT + j]);
        }
      } else {
        for (int e = lane; e < 16 * r; e += 64) {
          const int xr = e / r, j = e - xr * r;
          dst[e] = make_float2(out[xr * OP + j], out[xr * OP + RT + j]);
        }
      }
      __builtin_amdgcn_wave_barrier();  // read before the next tile overwrites it
    }
  }
}

// gradient fold, general masks: per location and coil,
//   K_c(loc,:) = sum_{(k,e) at loc} (W_c(loc,:) b_k - y_{k,c}(e)) conj(b_k)
// FS adjacent lanes share a location and take every FS-th of its (frame,
// sample) pairs; their partial sums meet by DPP at the end.  The pair counts
// reach q at the centre of k-space (every spoke passes there) and are a few
// at the edge, so splitting each location's list shortens the longest chain
// of dependent loads by FS.
constexpr int FOLD_FS = 4;  // lanes per location
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_fold_index2(FoldArgs a) {
  // B (every frame's b, q <= 128) staged once per workgroup, rows at an odd
  // stride so that the frames read by the lanes of one instruction fall in
  // different LDS banks; a lane's pairs and their data are loaded in batches
  // of PB, all of a batch's loads in flight together
  constexpr int PB = 8, FS = FOLD_FS, RTP = RT + 1;
  __shared__ float2 sB[128 * RTP];
  const int tid = threadIdx.x, sub = tid % FS;
  const int loc = blockIdx.x * (AG_NT / FS) + tid / FS, c = blockIdx.y;
  const int r = a.r;
  for (int e = tid; e < a.max_pairs * RT; e += AG_NT) {
    const int k = e / RT, j = e - k * RT;
    sB[k * RTP + j] = (j < r) ? a.B[(long)k * r + j] : make_float2(0.f, 0.f);
  }
  const int lc = min(loc, a.n - 1);
  const long base = ((long)c * a.n + lc) * r;
  float2 w[RT], kk[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    w[i] = (i < r) ? a.W[base + i] : make_float2(0.f, 0.f);
    kk[i] = make_float2(0.f, 0.f);
  }
  const int p0 = a.loc_ptr[lc], p1 = a.loc_ptr[lc + 1];
  __syncthreads();
  if (halted(a.st, a.check_halt)) return;
  const float2* yc = a.y + (long)c * a.m_max;
  const long ystride = (long)a.nc * a.m_max;
  for (int pb = p0 + sub; pb < p1; pb += PB * FS) {
    int2 ke[PB];
#pragma unroll
    for (int t = 0; t < PB; ++t) ke[t] = a.pairs[min(pb + FS * t, p1 - 1)];
    float2 yv[PB];
#pragma unroll
    for (int t = 0; t < PB; ++t) yv[t] = yc[ke[t].x * ystride + ke[t].y];
#pragma unroll
    for (int t = 0; t < PB; ++t) {
      if (pb + FS * t < p1) {
        const float2* bb = sB + ke[t].x * RTP;
        float2 res = make_float2(-yv[t].x, -yv[t].y);
#pragma unroll
        for (int i = 0; i < RT; ++i) res = cfma(res, w[i], bb[i]);
#pragma unroll
        for (int j = 0; j < RT; ++j) kk[j] = cfmaj(kk[j], res, bb[j]);
      }
    }
  }
  // the FS lanes of a location are all active here (they leave the loop
  // above at different times but reconverge); sum over them, then lane
  // `sub` stores columns j = sub, sub + FS, ...
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    kk[j].x += dpp_getf<DPP_XOR1>(kk[j].x);
    kk[j].y += dpp_getf<DPP_XOR1>(kk[j].y);
    kk[j].x += dpp_getf<DPP_XOR2>(kk[j].x);
    kk[j].y += dpp_getf<DPP_XOR2>(kk[j].y);
  }
  if (loc >= a.n) return;
#pragma unroll
  for (int j = 0; j < RT; ++j)
    if (j < r && j % FS == sub) a.K[base + j] = kk[j];
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

// coil maps in the layout the transforms read: [c][x / txx][y][x % txx], so
// that a workgroup's txx columns are one contiguous block per coil
__global__ void k_coil_block(const float2* coils, float2* dst, int nx, int ny, int txx, long n, int nc) {
  const long tot = n * nc;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long c = e / n, rem = e - c * n;
    const long xg = rem / ((long)ny * txx), rem2 = rem - xg * ny * txx;
    const int y = (int)(rem2 / txx), xl = (int)(rem2 - (long)y * txx);
    dst[e] = coils[c * n + (long)y * nx + xg * txx + xl];
  }
}

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
  else {
    // the x pass: grid_x (coil, ky) rows, a.txx of them per workgroup side
    // by side as the transform's columns (at most CT columns)
    BasisArgs b = a;
    int tyy = 1;
    while (2 * tyy * a.r <= CT && grid_x % (2 * tyy) == 0) tyy *= 2;
    b.txx = tyy;
    const dim3 gr((unsigned)(grid_x / tyy), grid_y);
    if (which == 2) hipLaunchKernelGGL((k_basis_rows<N, CT, false>), gr, dim3(AG_NT), 0, s, b);
    else hipLaunchKernelGGL((k_basis_rows<N, CT, true>), gr, dim3(AG_NT), 0, s, b);
  }
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

template <int N, int CT>
static void launch_adj_qr_n(const BasisArgs& a, hipStream_t s) {
  const dim3 g(a.nx), b(512);
  switch ((4 * a.r + 15) / 16) {  // row tiles of the [U G] embedding
    case 1: hipLaunchKernelGGL((k_adj_qr<N, CT, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_adj_qr<N, CT, 2>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_adj_qr<N, CT, 3>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_adj_qr<N, CT, 4>), g, b, 0, s, a); break;
  }
}

// one workgroup per image column; N in {64, 128, 256} and r <= 16
hipError_t launch_adj_qr(int N, const BasisArgs& a, hipStream_t s) {
  if (a.r < 1 || a.r > 16 || !a.qpart) return hipErrorInvalidValue;
  switch (N) {
    case 64: launch_adj_qr_n<64, 64>(a, s); break;
    case 128: launch_adj_qr_n<128, 32>(a, s); break;
    case 256: launch_adj_qr_n<256, 16>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fold2(const FoldArgs& a, bool lines, int grid_x, int grid_y, hipStream_t s) {
  const dim3 g(grid_x, grid_y);
  if (lines) {
    // the matrix-core fold needs whole 16-row tiles of x, at most four per
    // wave; its LDS holds b_p and the B operand for max_pairs pairs
    const int rt = a.r <= 8 ? 8 : 16;
    const size_t lds = sizeof(float2) * a.max_pairs * rt + sizeof(float) * (2 * rt + 2 * a.max_pairs + 4) * 2 * rt;
    static bool attr_set = false;  // q = 128 at rank 16 needs more than the default 64 KiB
    if (!attr_set) {
      hipError_t e1 = hipFuncSetAttribute((const void*)k_fold_lines_mma<8>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
      hipError_t e2 = hipFuncSetAttribute((const void*)k_fold_lines_mma<16>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
      if (e1 != hipSuccess) return e1;
      if (e2 != hipSuccess) return e2;
      attr_set = true;
    }
    if (a.nx >= 16 && a.nx <= 256 && a.r <= 8) hipLaunchKernelGGL(k_fold_lines_mma<8>, g, dim3(AG_NT), lds, s, a);
    else if (a.nx >= 16 && a.nx <= 256) hipLaunchKernelGGL(k_fold_lines_mma<16>, g, dim3(AG_NT), lds, s, a);
    else if (a.r <= 4) hipLaunchKernelGGL(k_fold_lines2<4>, g, dim3(AG_NT), 0, s, a);
    else if (a.r <= 8) hipLaunchKernelGGL(k_fold_lines2<8>, g, dim3(AG_NT), 0, s, a);
    else hipLaunchKernelGGL(k_fold_lines2<16>, g, dim3(AG_NT), 0, s, a);
  } else {
    // AG_NT / FOLD_FS locations per workgroup (grid_x is not used here)
    const dim3 gi((unsigned)((a.n + AG_NT / FOLD_FS - 1) / (AG_NT / FOLD_FS)), grid_y);
    if (a.r <= 4) hipLaunchKernelGGL(k_fold_index2<4>, gi, dim3(AG_NT), 0, s, a);
    else if (a.r <= 8) hipLaunchKernelGGL(k_fold_index2<8>, gi, dim3(AG_NT), 0, s, a);
    else if (a.r <= 12) hipLaunchKernelGGL(k_fold_index2<12>, gi, dim3(AG_NT), 0, s, a);
    else hipLaunchKernelGGL(k_fold_index2<16>, gi, dim3(AG_NT), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace ag
