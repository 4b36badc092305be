// The LS step of Algorithm 2 on the matrix cores: per-frame Gram
// G_k = (A_k U)^H (A_k U) and right-hand side h_k = (A_k U)^H y_k, then the
// batched r x r Cholesky solves b_k = G_k^{-1} h_k.
//
// Complex contractions run as real ones on MFMA: with the K sample rows of
// W (the coil-weighted, transformed basis at the sampled k-space positions)
// embedded as the real K x 2r matrix A = [Re W, Im W],
//   A^T A  gives  Re P = C[i][j] + C[r+i][r+j],  Im P = C[i][r+j] - C[r+i][j],
// and with B = [Re y_1..y_8, Im y_1..y_8] (8 samples' data as 16 columns)
//   A^T B  gives  Re h_{p,j} = C[j][p] + C[r+j][8+p], Im h_{p,j} = C[j][8+p] - C[r+j][p].
// Each 16x16 output tile is one v_mfma_*_16x16x4 accumulator (4 rows of K
// per instruction); the A operand is shared by the P tile and every h tile.
// FP32 MFMA for the plain form, FP64 MFMA for the mixed form.
#include <algorithm>

#include "kernels_core.hpp"
#include "mma.hpp"

namespace ag {


// ---------------------------------------------------------------------------
// 1D Cartesian: one workgroup (4 waves) per (sampled line u, tile t of 8 of
// its samples, coil group g).  Tile 0 also forms the line's Gram P_u.
// Rows of K are (c, x) for the group's coils; wave w takes rows x = 16s+4w..+3.
// Loads are unconditional (clamped address, then a select) so the MFMA chain
// is branch-free.  Outputs (FP64): Ppart[g][u][i][j], hpart[g][pair][j].
// ---------------------------------------------------------------------------
template <typename T, int TR, int UN, bool WP, int NWG>
__device__ __forceinline__ void gram_lines_loop(const GramLinesArgs& a, int u, int c0, int c1, int np, int pp,
                                                bool pok, int lane, int wave, int wg,
                                                typename Mma<T>::V (&P)[TR][TR], typename Mma<T>::V (&H)[TR]) {
  using M = Mma<T>;
  const int r = a.r, nx = a.nx, col = lane & 15, kk = lane >> 4;
  const int xl = 4 * wave + kk;
  int wj[TR], wim[TR];
  float wmask[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = 16 * t + col;
    const bool ok = i < 2 * r;
    wmask[t] = ok ? 1.f : 0.f;
    wj[t] = ok ? ((i < r) ? i : i - r) : 0;
    wim[t] = (i >= r) && ok;
  }
  const int yim = col >> 3;
  const float ymask = pok ? 1.f : 0.f;
  const float* Wf = reinterpret_cast<const float*>(a.W);
  // the item's data: [c][x][8 samples] complex (zero past the line's count)
  const float* Yitem = reinterpret_cast<const float*>(a.yg);
  // one flat loop over (coil, block of 16*UN rows x), the NWG groups of 4
  // waves taking every NWG-th block; the next block's operands are loaded
  // while the current one feeds the matrix cores
  constexpr int XB = 16 * UN;
  const int nxb = (nx + XB - 1) / XB;
  const int niter = max(0, c1 - c0) * nxb;
  T av[UN][TR], bv[UN];
  auto load = [&](int c, int x0, T (&A)[UN][TR], T (&Bv)[UN]) {
    const float* yrow = Yitem + 16L * ((long)c * nx) + 2 * (col & 7) + yim;
    const long wbase = 2L * (((long)c * a.ua + u) * nx * r);
#pragma unroll
    for (int q2 = 0; q2 < UN; ++q2) {
      // always load (from a clamped, valid address) and scale by a 0/1 mask,
      // so that no load sits under a branch
      const int x = x0 + 16 * q2 + xl;
      const float rm = (x < nx) ? 1.f : 0.f;
      const int xc = min(x, nx - 1);
#pragma unroll
      for (int t = 0; t < TR; ++t)
        A[q2][t] = (T)(Wf[wbase + 2L * (r * xc + wj[t]) + wim[t]] * (rm * wmask[t]));
      Bv[q2] = (T)(yrow[16 * xc] * (rm * ymask));
    }
  };
  // common shapes (every row block full, 2r filling the row tiles): a
  // wave-uniform base per step and a fixed per-lane offset, no masks (the
  // item's data is already zero past the line's count); a mask applied to a
  // loaded value would make the load wait at once
  const bool fast = (nx % XB) == 0 && 2 * r == 16 * TR;
  const float* Wline = Wf + 2L * ((long)u * nx * r);  // line u of coil 0
  const long CS = 2L * a.ua * nx * r;                 // coil stride of W, floats
  int lw[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) lw[t] = 2 * (r * xl + wj[t]) + wim[t];
  const int ly = 16 * xl + 2 * (col & 7) + yim;
  auto load_fast = [&](int c, int x0, T (&A)[UN][TR], T (&Bv)[UN]) {
    const float* wp = Wline + (long)c * CS + 2L * r * x0;
    const float* yp = Yitem + 16L * ((long)c * nx + x0);
#pragma unroll
    for (int q2 = 0; q2 < UN; ++q2) {
#pragma unroll
      for (int t = 0; t < TR; ++t) A[q2][t] = (T)wp[32 * r * q2 + lw[t]];
      Bv[q2] = (T)yp[256 * q2 + ly];
    }
  };
  {
    if (fast) {
      // the loads of DS steps are issued together, then their products run
      // (a step past the end loads a valid block of the last coil and skips
      // its products), so a workgroup waits for memory once per DS steps.
      // The group index is wave-uniform: in a scalar register, the step
      // counters and base addresses are scalar too.  DS measured per type.
      constexpr int DS = sizeof(T) == 8 ? GRAM_DS64 : GRAM_DS32;
      const int wgu = __builtin_amdgcn_readfirstlane(wg);
      int ci = wgu / nxb, xb = wgu % nxb;  // (coil, row block) of the next step to load
      for (int it0 = wgu; it0 < niter; it0 += DS * NWG) {
        T A[DS][UN][TR], Bv[DS][UN];
#pragma unroll
        for (int s2 = 0; s2 < DS; ++s2) {
          load_fast(min(c0 + ci, c1 - 1), xb * XB, A[s2], Bv[s2]);
          xb += NWG;
          while (xb >= nxb) {
            xb -= nxb;
            ++ci;
          }
        }
#pragma unroll
        for (int s2 = 0; s2 < DS; ++s2) {
          if (it0 + s2 * NWG < niter) {
#pragma unroll
            for (int q2 = 0; q2 < UN; ++q2) {
              if constexpr (WP) {
#pragma unroll
                for (int i = 0; i < TR; ++i)
#pragma unroll
                  for (int j = 0; j < TR; ++j) P[i][j] = M::mma(A[s2][q2][i], A[s2][q2][j], P[i][j]);
              }
#pragma unroll
              for (int i = 0; i < TR; ++i) H[i] = M::mma(A[s2][q2][i], Bv[s2][q2], H[i]);
            }
          }
        }
      }
      return;
    }
  }
  if (wg < niter) load(c0 + wg / nxb, (wg % nxb) * XB, av, bv);
  for (int it = wg; it < niter; it += NWG) {
    T an[UN][TR], bn[UN];
    const int itn = it + NWG;
    if (itn < niter) load(c0 + itn / nxb, (itn % nxb) * XB, an, bn);
#pragma unroll
    for (int q2 = 0; q2 < UN; ++q2) {
      if constexpr (WP) {
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int j = 0; j < TR; ++j) P[i][j] = M::mma(av[q2][i], av[q2][j], P[i][j]);
      }
#pragma unroll
      for (int i = 0; i < TR; ++i) H[i] = M::mma(av[q2][i], bv[q2], H[i]);
    }
#pragma unroll
    for (int q2 = 0; q2 < UN; ++q2) {
      bv[q2] = bn[q2];
#pragma unroll
      for (int t = 0; t < TR; ++t) av[q2][t] = an[q2][t];
    }
  }
}

// the Gram kernel's data per work item: [item][c][x][8 samples] complex,
// zero past the line's sample count (consecutive lanes read consecutive
// floats).  Grid (items bound, nc).
__global__ void k_build_yg(const float2* yu, const int4* items, int nc, int nx, float2* yg, const DevState* st) {
  const int w = blockIdx.x, c = blockIdx.y;
  if (st->err || w >= st->n_gwork) return;
  const int4 it = items[w];  // (line, tile, first pair, pair count)
  const float2* src = yu + (long)nc * nx * it.z + (long)c * it.w * nx;  // the line's [c][p][x] block
  float2* dst = yg + ((long)w * nc + c) * nx * 8;
  for (int e = threadIdx.x; e < nx * 8; e += blockDim.x) {
    const int x = e >> 3, p = 8 * it.y + (e & 7);
    dst[e] = (p < it.w) ? src[(long)p * nx + x] : make_float2(0.f, 0.f);
  }
}

// the Gram kernel's work items (line u, sample tile t), one block of 1024
// threads at setup: every sampled line contributes ceil(np_u / 8) items.
// Also the fold's dispatch order: the sampled lines by pair count, largest
// first (ties by index), then the unsampled rows in order, so that the
// longest fold workgroups start first instead of ending the launch.
__global__ __launch_bounds__(1024) void k_gram_work(const int2* unit_span, int4* items, int4* line_order,
                                                    int n_loc, DevState* st) {
  __shared__ int s_off[1024];
  __shared__ int s_np[1024];
  const int tid = threadIdx.x, nu = st->n_units;
  int cnt = 0;
  const int per = (nu + 1023) / 1024;
  for (int u = tid * per; u < min(nu, (tid + 1) * per); ++u) cnt += max(1, (unit_span[u].y + 7) / 8);
  s_off[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
    const int v = (tid >= off) ? s_off[tid - off] : 0;
    __syncthreads();
    s_off[tid] += v;
    __syncthreads();
  }
  int o = s_off[tid] - cnt;
  for (int u = tid * per; u < min(nu, (tid + 1) * per); ++u) {
    const int2 sp = unit_span[u];
    const int nt = max(1, (sp.y + 7) / 8);
    for (int t = 0; t < nt; ++t) items[o++] = make_int4(u, t, sp.x, sp.y);
  }
  if (tid == 1023) st->n_gwork = s_off[1023];
  if (nu <= 1024) {
    if (tid < nu) s_np[tid] = unit_span[tid].y;
    __syncthreads();
    if (tid < nu) {
      const int m = s_np[tid];
      int rk = 0;
      for (int v = 0; v < nu; ++v) rk += (s_np[v] > m) || (s_np[v] == m && v < tid);
      const int2 sp = unit_span[tid];
      line_order[rk] = make_int4(tid, sp.x, sp.y, 0);
    }
    for (int u = nu + tid; u < n_loc; u += 1024) line_order[u] = make_int4(u, 0, 0, 0);
  } else {
    for (int u = tid; u < n_loc; u += 1024) line_order[u] = make_int4(u, u < nu ? unit_span[u].x : 0, u < nu ? unit_span[u].y : 0, 0);
  }
}

template <typename T, int TR, int UN, int NWG>
__global__ __launch_bounds__(256 * NWG) void k_gram_lines_mma(GramLinesArgs a) {
  using M = Mma<T>;
  __shared__ T red[(TR * TR + TR) * 256];
  const int g = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wl = wave & 3, wg = wave >> 2;
  // the first item is requested together with the state (the list holds
  // gridDim.x entries at least; one past the count is not used)
  const int4 first = a.items[blockIdx.x];
  if (halted(a.st, a.check_halt)) return;
  const int nwork = a.st->n_gwork;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
  if (w > blockIdx.x) __syncthreads();  // the previous item's LDS reductions are complete
  const int4 item = (w == blockIdx.x) ? first : a.items[w];
  const int u = item.x, t = item.y;
  const int r = a.r, col = lane & 15;
  const int p0 = item.z, np = item.w;
  const int c0 = g * a.cg, c1 = min(a.nc, c0 + a.cg);
  // this lane's sample (B column) in tile t
  const int pl = 8 * t + (col & 7);
  const bool pok = pl < np;
  const int pp = pok ? pl : 0;
  GramLinesArgs al = a;
  al.yg = a.yg + (long)w * a.nc * a.nx * 8;  // this item's [c][x][8] block
  typename M::V P[TR][TR], H[TR];
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    H[i] = M::zero();
#pragma unroll
    for (int j = 0; j < TR; ++j) P[i][j] = M::zero();
  }
  if (t == 0)
    gram_lines_loop<T, TR, UN, true, NWG>(al, u, c0, c1, np, pp, pok, lane, wl, wg, P, H);
  else
    gram_lines_loop<T, TR, UN, false, NWG>(al, u, c0, c1, np, pp, pok, lane, wl, wg, P, H);
  // reduce across the 4 waves and form the complex outputs
  T* Pt = red;                    // TR*TR tiles
  T* Ht = red + TR * TR * 256;    // TR tiles of the h column block
  auto C = [&](const T* base, int ntile_cols, int i, int j) -> double {
    return (double)base[((i / 16) * ntile_cols + (j / 16)) * 256 + (i % 16) * 16 + (j % 16)];
  };
  constexpr int NTP = TR * TR + TR;
  __shared__ T scr[4 * NWG * NTP * 256];
  if (t == 0) {  // the P tiles and the h tiles together (red holds P, then h)
    typename M::V all[NTP];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      all[TR * TR + i] = H[i];
#pragma unroll
      for (int j = 0; j < TR; ++j) all[i * TR + j] = P[i][j];
    }
    tiles_reduce_par<T, 4 * NWG, NTP>(red, scr, all, wave, lane);
    double2* Pout = a.P + ((long)g * a.ua + u) * r * r;
    for (int e = tid; e < r * r; e += 256 * NWG) {
      const int i = e / r, j = e % r;
      const double re = C(Pt, TR, i, j) + C(Pt, TR, r + i, r + j);
      const double im = C(Pt, TR, i, r + j) - C(Pt, TR, r + i, j);
      Pout[e] = make_double2(re, im);
    }
  } else {
    tiles_reduce_par<T, 4 * NWG, TR>(Ht, scr, H, wave, lane);
  }
  const int npt = min(8, np - 8 * t);
  for (int e = tid; e < npt * r; e += 256 * NWG) {
    const int p = e / r, j = e % r;
    // rows j and r + j of the TR x 1 column of tiles, columns p (Re y) and 8 + p (Im y)
    const double re = C(Ht, 1, j, p) + C(Ht, 1, r + j, 8 + p);
    const double im = C(Ht, 1, j, 8 + p) - C(Ht, 1, r + j, p);
    a.hp[((long)g * a.npairs + p0 + 8 * t + p) * r + j] = make_double2(re, im);
  }
  }
}

// ---------------------------------------------------------------------------
// general masks: one workgroup per (frame k, chunk of its samples, coil c);
// rows of K are the chunk's samples for that coil.  A row of A is the W row
// as stored, Re W_0, Im W_0, Re W_1, .. (2r floats), then the sample's
// Re y, Im y (2r + 2 columns, padded to TR tiles of 16), so that one
// symmetric product A^T A carries the Gram and the right-hand side
// together; only its upper tiles (ti <= tj) are formed.
//   Re G_ij = C[2i][2j] + C[2i+1][2j+1],   Im G_ij = C[2i][2j+1] - C[2i+1][2j]
//   Re h_j  = C[2j][2r] + C[2j+1][2r+1],   Im h_j  = C[2j][2r+1] - C[2j+1][2r]
// Output part[k][chunk][c][r*r + r] (G entries, then h).
// Workgroups are dealt to the eight XCDs in turn by their linear index, and
// the index is laid out so that coil c runs on XCD c % 8: each XCD's L2 then
// holds the transformed basis of one coil (n r complex values), which every
// frame sampling a location gathers again.
// ---------------------------------------------------------------------------
template <int TR>
__device__ __forceinline__ constexpr int utile(int ti, int tj) { return ti * TR - ti * (ti - 1) / 2 + (tj - ti); }

constexpr int GRAM_XCDS = 8;

template <typename T, int TR>
__global__ __launch_bounds__(256) void k_gram_index_mma(GramIndexArgs a) {
  using M = Mma<T>;
  constexpr int NT = TR * (TR + 1) / 2;
  // the four waves' tiles, then (in wave 0's place) their sum: each sum
  // entry is written by the thread that read its four terms
  __shared__ T scr[4 * NT * 256];
  T* const red = scr;
  const int ncg = (a.nc + GRAM_XCDS - 1) / GRAM_XCDS;
  int bid = blockIdx.x;
  const int xg = bid % GRAM_XCDS;
  bid /= GRAM_XCDS;
  const int c = (bid % ncg) * GRAM_XCDS + xg;
  bid /= ncg;
  const int ch = bid % a.nchunks, k = bid / a.nchunks;
  if (c >= a.nc) return;  // padding of the coil count to a multiple of 8
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (halted(a.st, a.check_halt)) return;
  const int r = a.r, col = lane & 15, kk = lane >> 4;
  const int mk = a.m_k[k];
  const int i0 = ch * a.chunk, i1 = min(mk, i0 + a.chunk);
  const int ns = max(0, i1 - i0);
  // batches of 32 samples, batch j taken by wave j % 4; in a batch, lane
  // row kk of step u (4 rows per matrix-core step) is sample 8 kk + u, so
  // that a lane's 8 sample locations are adjacent in LDS
  constexpr int UB = 8;  // a multiple of 4 dividing GRAM_INDEX_CHUNK / 4
  const int nbat = (ns + 4 * UB - 1) / (4 * UB);
  typename M::V P[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) P[t] = M::zero();
  // the chunk's samples staged once: their W row offsets (location x 2r
  // floats, in bytes), so that the W gathers of a batch of steps do not wait on their
  // index loads, and their data y; padded to whole batches with location 0
  // (a valid address) and zero data
  __shared__ __align__(16) int s_loc[GRAM_INDEX_CHUNK];
  __shared__ float s_y[2 * GRAM_INDEX_CHUNK];
  const float2* const yck = a.y + ((long)k * a.nc + c) * a.m_max + i0;
  for (int e = tid; e < nbat * 4 * UB; e += 256) {
    const bool ok = e < ns;
    const int loc = a.mask[(long)k * a.m_max + i0 + min(e, max(ns - 1, 0))];
    const float2 yv = yck[min(e, max(ns - 1, 0))];
    s_loc[e] = ok ? loc * 8 * r : 0;
    s_y[2 * e] = ok ? yv.x : 0.f;
    s_y[2 * e + 1] = ok ? yv.y : 0.f;
  }
  __syncthreads();
  // every load of a batch is issued before its matrix-core work; each lane
  // loads from a valid address and padding and rows past the end are zeroed
  // by a select
  // (32-bit byte offsets from one base: the loads take the base from
  // scalar registers and do no 64-bit address arithmetic)
  const char* const Wc = reinterpret_cast<const char*>(a.W + (long)c * a.n * r);
  // this lane's column of A in each tile, i = 16 t + col: float i of the W
  // row (i < 2r), float i - 2r of the y sample (i = 2r, 2r + 1) or padding
  int wi[TR], yi[TR];
  bool isy[TR], used[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = 16 * t + col;
    used[t] = i < 2 * r + 2;
    isy[t] = used[t] && i >= 2 * r;
    wi[t] = i < 2 * r ? 4 * i : 0;  // bytes
    yi[t] = isy[t] ? i - 2 * r : 0;
  }
  for (int bj = wave; bj < nbat; bj += 4) {
    const int s0 = 4 * UB * bj + UB * kk;
    int lw[UB];
#pragma unroll
    for (int q4 = 0; q4 < UB / 4; ++q4) {
      const int4 l = *reinterpret_cast<const int4*>(s_loc + s0 + 4 * q4);
      lw[4 * q4] = l.x;
      lw[4 * q4 + 1] = l.y;
      lw[4 * q4 + 2] = l.z;
      lw[4 * q4 + 3] = l.w;
    }
    float v[UB][TR], yv[UB][TR];
    bool rv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      rv[u] = s0 + u < ns;
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        v[u][t] = *reinterpret_cast<const float*>(Wc + (unsigned)(lw[u] + wi[t]));
        yv[u][t] = s_y[2 * (s0 + u) + yi[t]];
      }
    }
    // empty asm statements that take every loaded value, after all the
    // batch's loads: without them the compiler moves each load under its
    // select's condition below, where it is then waited for on its own
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int t = 0; t < TR; ++t) asm volatile("" : "+v"(v[u][t]), "+v"(yv[u][t]));
    T av[UB][TR];
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int t = 0; t < TR; ++t) av[u][t] = (rv[u] && used[t]) ? (T)(isy[t] ? yv[u][t] : v[u][t]) : (T)0;
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int ti = 0; ti < TR; ++ti)
#pragma unroll
        for (int tj = ti; tj < TR; ++tj) P[utile<TR>(ti, tj)] = M::mma(av[u][ti], av[u][tj], P[utile<TR>(ti, tj)]);
  }
  tiles_reduce_par<T, 4, NT>(red, scr, P, wave, lane);
  // C[i][j] of the full symmetric product from its upper tiles
  auto C = [&](int i, int j) -> double {
    const int ti = i / 16, tj = j / 16;
    return ti <= tj ? (double)red[utile<TR>(ti, tj) * 256 + (i % 16) * 16 + (j % 16)]
                    : (double)red[utile<TR>(tj, ti) * 256 + (j % 16) * 16 + (i % 16)];
  };
  double2* out = a.part + (((long)k * a.nchunks + ch) * a.nc + c) * (r * r + r);
  for (int e = tid; e < r * r + r; e += 256) {
    if (e < r * r) {
      const int i = e / r, j = e % r;
      out[e] = make_double2(C(2 * i, 2 * j) + C(2 * i + 1, 2 * j + 1), C(2 * i, 2 * j + 1) - C(2 * i + 1, 2 * j));
    } else {
      const int j = e - r * r;
      out[e] = make_double2(C(2 * j, 2 * r) + C(2 * j + 1, 2 * r + 1), C(2 * j, 2 * r + 1) - C(2 * j + 1, 2 * r));
    }
  }
}

// ===========================================================================
// batched LS solve: b_k = G_k^{-1} h_k by Cholesky, one workgroup per frame;
// also cost_k = ||y_k||^2 - Re(h_k^H b_k).
// ===========================================================================
template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using T2 = float2;
  __device__ static T2 from(double2 v) { return d2f(v); }
  __device__ static T2 mul(T2 a, T2 b) { return cmul(a, b); }
  __device__ static T2 cjm(T2 a, T2 b) { return cjmul(a, b); }
  __device__ static T2 sub(T2 a, T2 b) { return csub(a, b); }
  __device__ static T2 scale(T2 a, float s) { return cscale(a, s); }
  static constexpr double tiny = 1e-5;  // pivot / max diagonal below this: cond(G) beyond FP32 use
};
template <>
struct Cx<double> {
  using T2 = double2;
  __device__ static T2 from(double2 v) { return v; }
  __device__ static T2 mul(T2 a, T2 b) { return dmul(a, b); }
  __device__ static T2 cjm(T2 a, T2 b) { return djmul(a, b); }
  __device__ static T2 sub(T2 a, T2 b) { return dsub(a, b); }
  __device__ static T2 scale(T2 a, double s) { return make_double2(a.x * s, a.y * s); }
  static constexpr double tiny = 1e-12;
};

template <typename T, int RT>
__global__ __launch_bounds__(SOLVE_NT) void k_solve(SolveArgs a) {
  using C = Cx<T>;
  using T2 = typename C::T2;
  __shared__ T2 G[16 * 16];
  __shared__ T2 h[16];
  __shared__ T2 z[16];
  __shared__ double2 part[SOLVE_NT];
  __shared__ int s_mk[512], s_po[512];
  const int k = blockIdx.x, tid = threadIdx.x, r = a.r;
  // requested before the state is read (valid addresses either way): the
  // frame's sample count and, for lines, its line and pair indices over the
  // whole padded width (entries past the frame's count are not used)
  const int mk = a.m_k[k];
  if (a.kind == 0) {
    for (int l = tid; l < a.width; l += SOLVE_NT) {
      s_mk[l] = a.unit_of[(long)k * a.width + l];  // sampled line of (k, l)
      s_po[l] = a.pair_of[(long)k * a.width + l];
    }
  }
  if (halted(a.st, a.check_halt)) return;
  const int E = r * r + r;  // G entries then h entries
  if (a.kind == 0) {
    const double2* const Pp = a.P;
    const double2* const Hp = a.hp;
    const long ua = a.ua, npairs = a.npairs;
    // sum over coil groups and the frame's lines; thread = (entry, slice of lines)
    const int L = mk / a.nx;
    __syncthreads();
    const int NS = max(1, SOLVE_NT / E), SW = SOLVE_NT / NS;
    for (int e0 = 0; e0 < E; e0 += SW) {
      const int e = e0 + tid % SW;
      const int sl = tid / SW;
      double2 s = make_double2(0.0, 0.0);
      const int items = a.ngroups * L;
      if (e < E && sl < NS && items > 0) {
        // the first MI items' loads issued together from clamped, valid
        // indices (the argument pointers in registers: a per-lane choice of
        // argument field would be a load), then summed in item order
        constexpr int MI = 8;
        const bool isP = e < r * r;
        const double2* const src = isP ? Pp : Hp;
        double2 vv[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          const int it = min(sl + i * NS, items - 1), gg = it / L, l = it - gg * L;
          vv[i] = src[isP ? ((long)gg * ua + s_mk[l]) * r * r + e : ((long)gg * npairs + s_po[l]) * r + (e - r * r)];
        }
#pragma unroll
        for (int i = 0; i < MI; ++i)
          if (sl + i * NS < items) s = dadd(s, vv[i]);
        for (int it = sl + MI * NS; it < items; it += NS) {
          const int gg = it / L, l = it - gg * L;
          s = dadd(s, src[isP ? ((long)gg * ua + s_mk[l]) * r * r + e : ((long)gg * npairs + s_po[l]) * r + (e - r * r)]);
        }
      }
      part[tid] = s;
      __syncthreads();
      if (tid < SW && e < E) {
        double2 t = part[tid];
        for (int q2 = 1; q2 < NS; ++q2) t = dadd(t, part[tid + q2 * SW]);
        if (e < r * r)
          G[(e / r) * 16 + (e % r)] = C::from(t);
        else
          h[e - r * r] = C::from(t);
      }
      __syncthreads();
    }
  } else {
    // sum over the frame's partials; thread = (entry, slice of partials)
    const int NS = max(1, SOLVE_NT / E), SW = SOLVE_NT / NS;
    const double2* const Pk = a.P + (long)k * a.nchunks * E;
    for (int e0 = 0; e0 < E; e0 += SW) {
      const int e = e0 + tid % SW;
      const int sl = tid / SW;
      double2 s = make_double2(0.0, 0.0);
      if (e < E && sl < NS) {
        constexpr int MI = 4;  // the first MI partials' loads issued together
        double2 vv[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) vv[i] = Pk[(long)min(sl + i * NS, a.nchunks - 1) * E + e];
#pragma unroll
        for (int i = 0; i < MI; ++i)
          if (sl + i * NS < a.nchunks) s = dadd(s, vv[i]);
        for (int ch = sl + MI * NS; ch < a.nchunks; ch += NS) s = dadd(s, Pk[(long)ch * E + e]);
      }
      part[tid] = s;
      __syncthreads();
      if (tid < SW && e < E) {
        double2 t = part[tid];
        for (int q2 = 1; q2 < NS; ++q2) t = dadd(t, part[tid + q2 * SW]);
        if (e < r * r)
          G[(e / r) * 16 + (e % r)] = C::from(t);
        else
          h[e - r * r] = C::from(t);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // the factorization and the two triangular solves: one wave, rows in lanes,
  // padded to RT with the identity
  if (tid >= 64) return;
  const int i = tid;
  T2 g[RT];
#pragma unroll
  for (int m = 0; m < RT; ++m)
    g[m] = (i < r && m < r) ? G[i * 16 + m] : T2{(T)(i == m ? 1 : 0), (T)0};
  double dmax = 0.0;
  for (int m = 0; m < r; ++m) dmax = fmax(dmax, (double)G[m * 16 + m].x);
  if (!wave_chol<T, T2, RT>(g, r, (T)(C::tiny * dmax))) {
    if (i == 0) set_error(a.st, 4 /*ENOTPD*/, k);
    return;
  }
  // L y = h, then L^H b = y; lane i ends with b_i
  T2 sv = (i < r) ? h[i] : T2{(T)0, (T)0};
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    const T2 yj = C::scale(lane_get(sv, j), (T)1 / lane_get(g[j].x, j));
    if (i == j) sv = yj;
    else if (i > j) sv = C::sub(sv, C::mul(g[j], yj));
  }
#pragma unroll
  for (int j = RT - 1; j >= 0; --j) {
    const T2 bj = C::scale(lane_get(sv, j), (T)1 / lane_get(g[j].x, j));
    if (i == j) sv = bj;
#pragma unroll
    for (int m = 0; m < j; ++m) {
      const T2 ljm = lane_get(g[m], j);  // L[j][m]
      if (i == m) sv = C::sub(sv, C::cjm(ljm, bj));
    }
  }
  double hb = 0.0;
  bool fin = true;
  if (i < r) {
    const T2 hi = h[i];
    hb = (double)hi.x * (double)sv.x + (double)hi.y * (double)sv.y;
    fin = isfinite((double)sv.x) && isfinite((double)sv.y);
    a.B[(long)k * r + i] = make_float2((float)sv.x, (float)sv.y);
    if (a.B_out) a.B_out[(long)k * r + i] = make_float2((float)sv.x, (float)sv.y);
    z[i] = sv;
  }
  hb = wave_sum(hb);
  const bool allfin = __all(fin);
  if (i == 0) {
    a.cost_k[k] = a.ysq_k[k] - hb;
    if (!allfin) set_error(a.st, 5 /*ENONFINITE*/, k);
  }
  if (a.kind == 0) {  // conj(b_k) at each of the frame's pairs
    wave_sync();
    const int L = mk / a.nx;
    for (int e = i; e < L * r; e += 64) {
      const int l = e / r, j = e - l * r;
      a.bcp[(long)s_po[l] * r + j] = make_float2((float)z[j].x, -(float)z[j].y);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int TR>
static void launch_lines_tr(const GramLinesArgs& a, int ny, int ngroups, int ht, hipStream_t s) {
  // about one work item per workgroup: every sampled line plus a few extra
  // sample tiles; a grid-stride loop takes any remainder
  (void)ht;
  const dim3 g(ny + 64, ngroups);
  constexpr int NWG = GRAM_NWG;
  if (a.nx >= 64) hipLaunchKernelGGL((k_gram_lines_mma<T, TR, 4, NWG>), g, dim3(256 * NWG), 0, s, a);
  else hipLaunchKernelGGL((k_gram_lines_mma<T, TR, 1, NWG>), g, dim3(256 * NWG), 0, s, a);
}

hipError_t launch_gram_work(const int2* unit_span, int4* items, int4* line_order, int n_loc, DevState* st,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_gram_work, dim3(1), dim3(1024), 0, s, unit_span, items, line_order, n_loc, st);
  return hipGetLastError();
}

hipError_t launch_gram_lines(const GramLinesArgs& a, int ny, int ngroups, int max_pairs, bool fp64,
                             hipStream_t s) {
  const int ht = std::max(1, (max_pairs + 7) / 8);
  const int tr = (2 * a.r + 15) / 16;
  if (fp64) {
    if (tr == 1) launch_lines_tr<double, 1>(a, ny, ngroups, ht, s);
    else launch_lines_tr<double, 2>(a, ny, ngroups, ht, s);
  } else {
    if (tr == 1) launch_lines_tr<float, 1>(a, ny, ngroups, ht, s);
    else launch_lines_tr<float, 2>(a, ny, ngroups, ht, s);
  }
  return hipGetLastError();
}

hipError_t launch_gram_index(const GramIndexArgs& a, int q, bool fp64, hipStream_t s) {
  const int tr = (2 * a.r + 2 + 15) / 16;  // W's 2r real columns and y's two
  const int ncg = (a.nc + GRAM_XCDS - 1) / GRAM_XCDS;
  const dim3 g((unsigned)q * a.nchunks * ncg * GRAM_XCDS);
  if (fp64) {
    if (tr == 1) hipLaunchKernelGGL((k_gram_index_mma<double, 1>), g, dim3(256), 0, s, a);
    else if (tr == 2) hipLaunchKernelGGL((k_gram_index_mma<double, 2>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_gram_index_mma<double, 3>), g, dim3(256), 0, s, a);
  } else {
    if (tr == 1) hipLaunchKernelGGL((k_gram_index_mma<float, 1>), g, dim3(256), 0, s, a);
    else if (tr == 2) hipLaunchKernelGGL((k_gram_index_mma<float, 2>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_gram_index_mma<float, 3>), g, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int q, bool fp64, hipStream_t s) {
  // the factor's register tile: rows padded to 8, 12 or 16 with the identity
  if (fp64) {
    if (a.r <= 8) hipLaunchKernelGGL((k_solve<double, 8>), dim3(q), dim3(SOLVE_NT), 0, s, a);
    else if (a.r <= 12) hipLaunchKernelGGL((k_solve<double, 12>), dim3(q), dim3(SOLVE_NT), 0, s, a);
    else hipLaunchKernelGGL((k_solve<double, 16>), dim3(q), dim3(SOLVE_NT), 0, s, a);
  } else {
    if (a.r <= 8) hipLaunchKernelGGL((k_solve<float, 8>), dim3(q), dim3(SOLVE_NT), 0, s, a);
    else if (a.r <= 12) hipLaunchKernelGGL((k_solve<float, 12>), dim3(q), dim3(SOLVE_NT), 0, s, a);
    else hipLaunchKernelGGL((k_solve<float, 16>), dim3(q), dim3(SOLVE_NT), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace ag

namespace ag {

// ===========================================================================
// Gram of the columns of [A B] over n pixel rows on MFMA (the QR step):
// real embedding [Re A, Re B, Im A, Im B] (2m columns, m = m1 + m2), upper
// 16x16 tiles only.  B may be the sum of nparts partial arrays (stride
// part_stride); with write_sum the summed B is stored back into part 0.
// Output: per block, the upper triangle (i <= j, tri order) of the complex
// m x m Gram, FP64.
// ===========================================================================
template <typename T, int TRM, int NSM>
__global__ __launch_bounds__(256 * NSM) void k_qr_gram_mma(GramColsArgs a) {
  using M = Mma<T>;
  constexpr int NT = TRM * (TRM + 1) / 2;
  constexpr int RC = TRM <= 4 ? 64 : 32;  // rows per chunk staged in LDS (fewer for wide Grams: registers)
  // row pitch of the staged real embedding: the 4 rows one MFMA step reads
  // land in disjoint quarters of the 64 LDS banks
  constexpr int LDX = (16 * TRM) % 64 == 0 || (16 * TRM) % 64 == 32 ? 16 * TRM + 16 : 16 * TRM;
  constexpr int EM = RC * 8 * TRM / 256;  // complex elements per thread per chunk (m <= 8 TRM)
  // NSM streams of 4 waves each take interleaved chunks of the block's rows
  __shared__ T X[NSM][RC * LDX];
  __shared__ T red[NT * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sm = wave >> 2, wl = wave & 3, lt = tid & 255;  // stream, its wave, its thread
  const int col = lane & 15, kk = lane >> 4;
  const int m1 = a.m1, m2 = a.m2, m = m1 + m2;
  const long pa = (long)blockIdx.x * a.rows_per_block;
  const long pb = min(a.n, pa + a.rows_per_block);
  for (int e = tid; e < NSM * RC * LDX; e += 256 * NSM) (&X[0][0])[e] = (T)0;  // columns >= 2m stay zero
  // this thread's elements of a chunk: e < RC*m1 from A, then RC*m2 from B,
  // both contiguous in the pixel-major arrays
  int erow[EM], ecol[EM];
#pragma unroll
  for (int q = 0; q < EM; ++q) {
    const int e = lt + 256 * q;
    if (e < RC * m1) {
      if (a.a_colmajor) {  // consecutive threads on consecutive rows of a column
        ecol[q] = e / RC;
        erow[q] = e - ecol[q] * RC;
      } else {
        erow[q] = e / m1;
        ecol[q] = e - erow[q] * m1;
      }
    } else if (e < RC * m) {
      const int f = e - RC * m1;
      erow[q] = f / m2;
      ecol[q] = m1 + (f - (f / m2) * m2);
    } else {
      erow[q] = RC;  // no element
      ecol[q] = 0;
    }
  }
  // the chunk at row p0: every load issued unconditionally from a clamped,
  // valid address into w (an A element loads its one entry four times, from
  // the cache), and the masks and the sum over B's partial arrays applied
  // only when the chunk is staged, so that the loads stay in flight during
  // the previous chunk's matrix-core work
  // (the arguments in registers: a per-lane choice between two argument
  // fields would otherwise be a load from the argument block)
  const float2* const pA = a.A;
  const float2* const pB = a.B;
  const long pstride = a.part_stride, ncol = a.n;
  const int nparts = a.nparts, colmaj = a.a_colmajor;
  float2 w[EM][4];
  auto load = [&](long p0) {
#pragma unroll
    for (int q = 0; q < EM; ++q) {
      const long p = min(p0 + min(erow[q], RC - 1), pb - 1);
      const bool isb = ecol[q] >= m1;
      const long off = isb ? p * m2 + (ecol[q] - m1) : (colmaj ? ecol[q] * ncol + p : p * m1 + ecol[q]);
      const float2* src = isb ? pB : pA;
#pragma unroll
      for (int g = 0; g < 4; ++g) w[q][g] = src[(isb ? min(g, nparts - 1) : 0) * pstride + off];
    }
  };
  typename M::V acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = M::zero();
  load(pa + sm * RC);
  // the state is read once the first chunk's loads are in flight
  if (halted(a.st, a.check_halt)) return;
  // every workgroup-wide step runs the same number of times in both streams
  for (long base = pa; base < pb; base += NSM * RC) {
    const long p0 = base + sm * RC;
    __syncthreads();  // the previous chunk's MFMA reads of X are done
    T* Xs = X[sm];
#pragma unroll
    for (int q = 0; q < EM; ++q) {
      // element q (zero for rows at or past pb): the A entry, or the sum
      // over B's partial arrays, in the order (0 + 1) + (2 + 3) + 4 + ...
      const long p = p0 + erow[q];
      const bool ok = erow[q] < RC && p < pb;
      const bool isb = ecol[q] >= m1;
      const float2 z = make_float2(0.f, 0.f);
      float2 v = cadd(cadd(w[q][0], (isb && nparts > 1) ? w[q][1] : z),
                      cadd((isb && nparts > 2) ? w[q][2] : z, (isb && nparts > 3) ? w[q][3] : z));
      if (ok && isb)
        for (int g0 = 4; g0 < nparts; ++g0)  // more than four partial arrays
          v = cadd(v, pB[g0 * pstride + p * m2 + (ecol[q] - m1)]);
      if (!ok) v = z;
      if (erow[q] < RC) {
        Xs[erow[q] * LDX + ecol[q]] = (T)v.x;
        Xs[erow[q] * LDX + m + ecol[q]] = (T)v.y;
        if (a.write_sum && nparts > 1 && isb && p < pb) const_cast<float2*>(pB)[p * m2 + (ecol[q] - m1)] = v;
      }
    }
    __syncthreads();
    if (base + NSM * RC < pb) load(p0 + NSM * RC);  // in flight during this chunk's MFMAs
#pragma unroll
    for (int st = 0; st < RC / 16; ++st) {  // each wave takes RC / 4 rows, 4 per MFMA step
      const T* xr = Xs + ((RC / 4) * wl + 4 * st + kk) * LDX + col;
      T xv[TRM];
#pragma unroll
      for (int t = 0; t < TRM; ++t) xv[t] = xr[16 * t];
#pragma unroll
      for (int i = 0; i < TRM; ++i)
#pragma unroll
        for (int j = i; j < TRM; ++j) {
          const int ti = i * TRM - i * (i - 1) / 2 + (j - i);
          acc[ti] = M::mma(xv[i], xv[j], acc[ti]);
        }
    }
  }
  if constexpr (4 * NSM * NT * 256 * sizeof(T) <= 48 * 1024) {
    __shared__ T scr[4 * NSM * NT * 256];
    tiles_reduce_par<T, 4 * NSM, NT>(red, scr, acc, wave, lane);
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) tile_reduce_n<T, 4 * NSM>(red + t * 256, acc[t], wave, lane);
  }
  // C(i, j) of the real 2m x 2m Gram from the upper tiles
  auto C = [&](int i, int j) -> double {
    if (i > j) {
      const int t = i;
      i = j;
      j = t;
    }
    const int a_ = i / 16, b_ = j / 16;
    const int ti = a_ * TRM - a_ * (a_ - 1) / 2 + (b_ - a_);
    return (double)red[ti * 256 + (i % 16) * 16 + (j % 16)];
  };
  const int nout = m * (m + 1) / 2;
  for (int o = tid; o < nout; o += 256 * NSM) {
    int i, j;
    tri_index(o, m, i, j);
    const double re = C(i, j) + C(m + i, m + j);
    const double imv = C(i, m + j) - C(m + i, j);
    if constexpr (sizeof(T) == 4)  // an FP32 Gram's partials carry FP32 information
      reinterpret_cast<float2*>(a.part)[(long)blockIdx.x * nout + o] = make_float2((float)re, (float)imv);
    else
      a.part[(long)blockIdx.x * nout + o] = make_double2(re, imv);
  }
}

// (three or four row tiles keep their accumulators with one stream of 256 threads)
hipError_t launch_qr_gram(const GramColsArgs& a, int nblk, bool fp64, hipStream_t s) {
  const int trm = (2 * (a.m1 + a.m2) + 15) / 16;
  const dim3 g(nblk);
  if (fp64) {
    switch (trm) {
      case 1: hipLaunchKernelGGL((k_qr_gram_mma<double, 1, QR_NSM>), g, dim3(256 * QR_NSM), 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_qr_gram_mma<double, 2, QR_NSM>), g, dim3(256 * QR_NSM), 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_qr_gram_mma<double, 3, 1>), g, dim3(256), 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_qr_gram_mma<double, 4, 1>), g, dim3(256), 0, s, a); break;
      // wider Grams (the spectral init's q columns, up to 48)
      case 5: hipLaunchKernelGGL((k_qr_gram_mma<double, 5, 1>), g, dim3(256), 0, s, a); break;
      case 6: hipLaunchKernelGGL((k_qr_gram_mma<double, 6, 1>), g, dim3(256), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (trm) {
      case 1: hipLaunchKernelGGL((k_qr_gram_mma<float, 1, QR_NSM>), g, dim3(256 * QR_NSM), 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_qr_gram_mma<float, 2, QR_NSM>), g, dim3(256 * QR_NSM), 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_qr_gram_mma<float, 3, 1>), g, dim3(256), 0, s, a); break;
      default: hipLaunchKernelGGL((k_qr_gram_mma<float, 4, 1>), g, dim3(256), 0, s, a); break;
    }
  }
  return hipGetLastError();
}

// upper tile ti of a TRM x TRM tile grid (row-major over the upper
// triangle): its tile row and column
constexpr int utile_row(int trm, int ti) {
  int i = 0;
  while (ti >= trm - i) {
    ti -= trm - i;
    ++i;
  }
  return i;
}
constexpr int utile_col(int trm, int ti) {
  int i = 0;
  while (ti >= trm - i) {
    ti -= trm - i;
    ++i;
  }
  return i + ti;
}

// one 4-row step of wave W's upper tiles W, W + 4, ... (the tile rows it
// reads and the accumulator it feeds fixed at compile time)
template <int TRM, int W, int K = 0>
__device__ __forceinline__ void init_gram_tiles(const double* xr, typename Mma<double>::V* acc) {
  constexpr int NTL = TRM * (TRM + 1) / 2, TI = W + 4 * K;
  if constexpr (TI < NTL) {
    constexpr int I = utile_row(TRM, TI), J = utile_col(TRM, TI);
    acc[K] = Mma<double>::mma(xr[16 * I], xr[16 * J], acc[K]);
    init_gram_tiles<TRM, W, K + 1>(xr, acc);
  }
}

template <int TRM, int W, int RC, int LDX>
__device__ __forceinline__ void init_gram_chunk(const double* X, int kk, int col, typename Mma<double>::V* acc) {
#pragma unroll
  for (int st = 0; st < RC / 4; ++st) init_gram_tiles<TRM, W>(X + (4 * st + kk) * LDX + col, acc);
}

// X0^H X0 of the spectral init (q <= 48 column-major FP32 columns of n
// pixels) on the f64 matrix cores, one workgroup per block of rows.  A chunk
// of RC rows is staged in LDS as the real embedding [Re X0 | Im X0] (FP64,
// odd row pitch: consecutive rows' 8-byte writes fall in distinct banks);
// wave w owns the upper tiles w, w + 4, ... over all of the chunk's rows, so
// no sum across waves is needed.  Each chunk's loads are in flight during
// the previous chunk's matrix-core work.  Output: the block's complex upper
// triangle (tri order, FP64) at part[blockIdx.x * nout].
template <int TRM>
__global__ __launch_bounds__(256) void k_init_gram(GramColsArgs a) {
  using M = Mma<double>;
  constexpr int NTL = TRM * (TRM + 1) / 2, TPW = (NTL + 3) / 4;
  constexpr int RC = 32, LDX = 16 * TRM + 1;
  constexpr int EM = (RC * 8 * TRM + 255) / 256;  // complex elements per thread per chunk (q <= 8 TRM)
  constexpr int XW = RC * LDX > NTL * 256 ? RC * LDX : NTL * 256;
  __shared__ double X[XW];  // the staged chunk, then the tiles
  const int tid = threadIdx.x, lane = tid & 63, col = lane & 15, kk = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = a.m1;
  const long n = a.n, pa = (long)blockIdx.x * a.rows_per_block, pb = min(n, pa + a.rows_per_block);
  const float2* const A = a.A;
  int erow[EM], ecol[EM];
#pragma unroll
  for (int i = 0; i < EM; ++i) {
    const int e = tid + 256 * i;
    const bool ok = e < RC * q;
    ecol[i] = ok ? e / RC : q;  // a column past q: no element
    erow[i] = ok ? e - (e / RC) * RC : 0;
  }
  float2 w[EM];
  auto load = [&](long p0) {  // valid, clamped addresses; rows past pb are zeroed when staged
#pragma unroll
    for (int i = 0; i < EM; ++i) w[i] = A[(long)min(ecol[i], q - 1) * n + min(p0 + erow[i], pb - 1)];
  };
  load(pa);
  for (int e = tid; e < XW; e += 256) X[e] = 0.0;  // columns from 2q on stay zero
  if (halted(a.st, a.check_halt)) return;
  M::V acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = M::zero();
  for (long base = pa; base < pb; base += RC) {
    __syncthreads();  // the previous chunk's reads (and the zero fill) are done
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const double re = base + erow[i] < pb ? (double)w[i].x : 0.0;
      const double im = base + erow[i] < pb ? (double)w[i].y : 0.0;
      if (ecol[i] < q) {
        X[erow[i] * LDX + ecol[i]] = re;
        X[erow[i] * LDX + q + ecol[i]] = im;
      }
    }
    __syncthreads();
    if (base + RC < pb) load(base + RC);
    switch (wave) {  // wave-uniform: each branch's tiles fixed at compile time
      case 0: init_gram_chunk<TRM, 0, RC, LDX>(X, kk, col, acc); break;
      case 1: init_gram_chunk<TRM, 1, RC, LDX>(X, kk, col, acc); break;
      case 2: init_gram_chunk<TRM, 2, RC, LDX>(X, kk, col, acc); break;
      default: init_gram_chunk<TRM, 3, RC, LDX>(X, kk, col, acc); break;
    }
  }
  __syncthreads();  // the last chunk's reads of X are done: X holds the tiles now
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int ti = wave + 4 * k;
    if (ti < NTL) {
#pragma unroll
      for (int v = 0; v < 4; ++v) X[ti * 256 + M::row(lane, v) * 16 + col] = acc[k][v];
    }
  }
  __syncthreads();
  auto C = [&](int i, int j) -> double {  // entry (i, j) of the real 2q x 2q Gram
    if (i > j) {
      const int t = i;
      i = j;
      j = t;
    }
    const int a_ = i / 16, b_ = j / 16;
    return X[(a_ * TRM - a_ * (a_ - 1) / 2 + (b_ - a_)) * 256 + (i % 16) * 16 + (j % 16)];
  };
  const int nout = q * (q + 1) / 2;
  double2* out = a.part + (long)blockIdx.x * nout;
  for (int o = tid; o < nout; o += 256) {
    int i, j;
    tri_index(o, q, i, j);
    out[o] = make_double2(C(i, j) + C(q + i, q + j), C(i, q + j) - C(q + i, j));
  }
}

// one 4-row step of wave W's complex tiles W, W + 8, ...: tile (a, b) of
// X0^H X0 is Re = Xr_a^T Xr_b + Xi_a^T Xi_b and Im = Xr_a^T Xi_b - Xi_a^T Xr_b
// (two accumulators, four matrix-core products per step)
template <int QT, int W, int K = 0>
__device__ __forceinline__ void init_gram_cx_tiles(const double* xr, const double* xi,
                                                   typename Mma<double>::V* acc) {
  constexpr int NCT = QT * (QT + 1) / 2, TI = W + 8 * K;
  if constexpr (TI < NCT) {
    constexpr int I = utile_row(QT, TI), J = utile_col(QT, TI);
    acc[2 * K] = Mma<double>::mma(xr[16 * I], xr[16 * J], acc[2 * K]);
    acc[2 * K] = Mma<double>::mma(xi[16 * I], xi[16 * J], acc[2 * K]);
    acc[2 * K + 1] = Mma<double>::mma(xr[16 * I], xi[16 * J], acc[2 * K + 1]);
    acc[2 * K + 1] = Mma<double>::mma(-xi[16 * I], xr[16 * J], acc[2 * K + 1]);
    init_gram_cx_tiles<QT, W, K + 1>(xr, xi, acc);
  }
}

template <int QT, int W, int RC, int LDX>
__device__ __forceinline__ void init_gram_cx_chunk(const double* X, int kk, int col, typename Mma<double>::V* acc) {
#pragma unroll
  for (int st = 0; st < RC / 4; ++st) {
    const double* xr = X + (4 * st + kk) * LDX + col;
    init_gram_cx_tiles<QT, W>(xr, xr + 16 * QT, acc);
  }
}

// X0^H X0 for 48 < q <= 128 columns (QT = ceil(q / 16) complex column
// tiles): 512 threads, a chunk of RC rows staged as [Re X0 | Im X0] in
// FP64 (odd pitch), wave w owning the complex upper tiles w, w + 8, ...; each
// wave writes its tiles' entries of the upper triangle straight to the
// block's partial (tri order), so no sum across waves is needed.
template <int QT>
__global__ __launch_bounds__(512) void k_init_gram_cx(GramColsArgs a) {
  using M = Mma<double>;
  constexpr int NCT = QT * (QT + 1) / 2, TPW = (NCT + 7) / 8;
  constexpr int RC = 32, LDX = 32 * QT + 1;
  constexpr int EM = (RC * 16 * QT + 511) / 512;  // complex elements per thread per chunk (q <= 16 QT)
  __shared__ double X[RC * LDX];
  const int tid = threadIdx.x, lane = tid & 63, col = lane & 15, kk = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = a.m1;
  const long n = a.n, pa = (long)blockIdx.x * a.rows_per_block, pb = min(n, pa + a.rows_per_block);
  const float2* const A = a.A;
  int erow[EM], ecol[EM];
#pragma unroll
  for (int i = 0; i < EM; ++i) {
    const int e = tid + 512 * i;
    const bool ok = e < RC * q;
    ecol[i] = ok ? e / RC : q;  // a column past q: no element
    erow[i] = ok ? e - (e / RC) * RC : 0;
  }
  float2 w[EM];
  auto load = [&](long p0) {
#pragma unroll
    for (int i = 0; i < EM; ++i) w[i] = A[(long)min(ecol[i], q - 1) * n + min(p0 + erow[i], pb - 1)];
  };
  load(pa);
  for (int e = tid; e < RC * LDX; e += 512) X[e] = 0.0;  // columns from q on stay zero
  if (halted(a.st, a.check_halt)) return;
  M::V acc[2 * TPW];
#pragma unroll
  for (int t = 0; t < 2 * TPW; ++t) acc[t] = M::zero();
  for (long base = pa; base < pb; base += RC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const double re = base + erow[i] < pb ? (double)w[i].x : 0.0;
      const double im = base + erow[i] < pb ? (double)w[i].y : 0.0;
      if (ecol[i] < q) {
        X[erow[i] * LDX + ecol[i]] = re;
        X[erow[i] * LDX + 16 * QT + ecol[i]] = im;
      }
    }
    __syncthreads();
    if (base + RC < pb) load(base + RC);
    switch (wave) {
      case 0: init_gram_cx_chunk<QT, 0, RC, LDX>(X, kk, col, acc); break;
      case 1: init_gram_cx_chunk<QT, 1, RC, LDX>(X, kk, col, acc); break;
      case 2: init_gram_cx_chunk<QT, 2, RC, LDX>(X, kk, col, acc); break;
      case 3: init_gram_cx_chunk<QT, 3, RC, LDX>(X, kk, col, acc); break;
      case 4: init_gram_cx_chunk<QT, 4, RC, LDX>(X, kk, col, acc); break;
      case 5: init_gram_cx_chunk<QT, 5, RC, LDX>(X, kk, col, acc); break;
      case 6: init_gram_cx_chunk<QT, 6, RC, LDX>(X, kk, col, acc); break;
      default: init_gram_cx_chunk<QT, 7, RC, LDX>(X, kk, col, acc); break;
    }
  }
  // this wave's tiles to the block's upper triangle: entry (i, j), i <= j < q,
  // at o = i q - i (i - 1) / 2 + (j - i)
  const int nout = q * (q + 1) / 2;
  double2* out = a.part + (long)blockIdx.x * nout;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int ti = wave + 8 * k;
    if (ti < NCT) {
      int ta = 0, rem = ti;
      while (rem >= QT - ta) {
        rem -= QT - ta;
        ++ta;
      }
      const int tb = ta + rem;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * ta + M::row(lane, v), j = 16 * tb + col;
        if (i <= j && j < q) out[i * q - i * (i - 1) / 2 + (j - i)] = make_double2(acc[2 * k][v], acc[2 * k + 1][v]);
      }
    }
  }
}

hipError_t launch_init_gram_cx(const GramColsArgs& a, int nblk, hipStream_t s) {
  if (a.m2 != 0 || !a.a_colmajor || a.m1 <= 48 || a.m1 > 128 || a.rows_per_block % 32 != 0)
    return hipErrorInvalidValue;
  const dim3 g(nblk), b(512);
  switch ((a.m1 + 15) / 16) {
    case 4: hipLaunchKernelGGL((k_init_gram_cx<4>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_init_gram_cx<5>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_init_gram_cx<6>), g, b, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_init_gram_cx<7>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_init_gram_cx<8>), g, b, 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_init_gram(const GramColsArgs& a, int nblk, hipStream_t s) {
  if (a.m2 != 0 || !a.a_colmajor || a.m1 < 1 || a.m1 > 48 || a.rows_per_block % 32 != 0) return hipErrorInvalidValue;
  const dim3 g(nblk), b(256);
  switch ((2 * a.m1 + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_init_gram<1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_init_gram<2>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_init_gram<3>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_init_gram<4>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_init_gram<5>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_init_gram<6>), g, b, 0, s, a); break;
  }
  return hipGetLastError();
}

// sum over nblk partials of nout FP64 entries, in workgroup-slice order:
// workgroup = 16 outputs x 16 slices of the partials, LDS tree over slices
__global__ __launch_bounds__(256) void k_sum_partials(const double2* part, int nblk, int nout, double2* out) {
  __shared__ double2 red[256];
  const int tid = threadIdx.x, ol = tid & 15, sl = tid >> 4;
  const int o = blockIdx.x * 16 + ol;
  double2 acc = make_double2(0.0, 0.0);
  if (o < nout) {
#pragma unroll 16
    for (int b = sl; b < nblk; b += 16) acc = dadd(acc, part[(long)b * nout + o]);
  }
  red[tid] = acc;
  __syncthreads();
  for (int off = 128; off >= 16; off >>= 1) {
    if (tid < off) red[tid] = dadd(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid < 16 && o < nout) out[o] = red[tid];
}

hipError_t launch_sum_partials(const double2* part, int nblk, int nout, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3((nout + 15) / 16), dim3(256), 0, s, part, nblk, nout, out);
  return hipGetLastError();
}

// dst[i] = sum_g src[g*stride + i] (partial gradients of the coil groups)
__global__ void k_sum_parts(const float2* src, long stride, int nparts, float2* dst, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long step = (long)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    float2 s = src[i];
    for (int g = 1; g < nparts; ++g) s = cadd(s, src[g * stride + i]);
    dst[i] = s;
  }
}

}  // namespace ag
