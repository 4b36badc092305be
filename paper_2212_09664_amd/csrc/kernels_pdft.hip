// The mixed form's phase-encode (ky) transforms for 1D Cartesian masks as
// dense partial DFTs on the matrix cores: FP16 operands split hi + lo,
// FP32 accumulation (v_mfma_f32_16x16x32_f16).
//
//   forward  W_c[u][col] = N^-1/2 sum_y exp(-2 pi i ky_u y / N) s_c(x, y) U(x, y, j)
//   adjoint  G[y][col]  += conj(s_c(x, y)) N^-1/2 sum_u exp(+2 pi i ky_u y / N) K_c[u][col]
//
// with col = x*r + j (the row-interleaved layouts of W, K and U) and u over
// the sampled k-space rows.  A complex product is embedded as a real GEMM
// over a doubled contraction index kappa = (part, y) (forward) or (part, u)
// (adjoint): part 0 carries cos, part 1 carries -+sin; the B operand holds
// (Re, -Im) for the real output tiles and (Im, Re) for the imaginary ones.
// Each operand a is split a = hi + lo with hi = fp16(a), lo = fp16(a - hi);
// the product keeps hi*hi + hi*lo + lo*hi.  The data operand is scaled by a
// power of two per workgroup (and per coil) so that its largest entry sits
// near 2^14, which keeps both halves in fp16's normal range.  DFT entries
// come from two LDS tables (part 0: cos, part 1: the signed sin), one word
// per entry holding its fp16 hi and lo halves, indexed by (ky*y) mod N; the
// hi and lo fragments are two byte permutations of eight such words.
//
// MFMA lane layout (16x16x32 f16, gfx950): lane l holds A[l%16][8(l/16)+e]
// and B[8(l/16)+e][l%16], e = 0..7; the result register v holds
// D[4(l/16)+v][l%16].
#include "kernels_core.hpp"

namespace ag {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_hl(float v, _Float16& h, _Float16& l) {
  h = (_Float16)v;
  l = (_Float16)(v - (float)h);
}

// power-of-two scale putting the largest magnitude near 2^14 (1 for zeros)
__device__ __forceinline__ float pow2_scale(float amax) {
  if (!(amax > 0.f) || !isfinite(amax)) return 1.f;
  int e;
  frexpf(amax, &e);  // amax in [2^(e-1), 2^e)
  return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ float block_max(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float m = 0.f;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
  return m;
}

// one DFT entry as a word: fp16 hi in the low half, fp16 lo in the high half
__device__ __forceinline__ uint32_t pack_hl(float v) {
  _Float16 h, l;
  split_hl(v, h, l);
  return (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
}

// the two halves of the contraction index: part 0 carries cos(2 pi t / N),
// part 1 carries psign * sin(2 pi t / N)
__device__ __forceinline__ void load_tables(uint32_t* t0, uint32_t* t1, const float2* tw, int N, float psign) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    const float2 w = tw[t];  // exp(-2 pi i t / N) = (cos, -sin)
    t0[t] = pack_hl(w.x);
    t1[t] = pack_hl(-psign * w.y);
  }
}

typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// LDS of both kernels, tables first: their byte offsets then fit the
// 16-bit immediate offset of an LDS read, so a lookup needs no base add
template <int N>
struct alignas(16) PdftLds {
  uint32_t tw0[N], tw1[N];
  int s_ky[N];
  float red[4];
  _Float16 D[4 * 32 * (N + 8)];
};

// eight table words -> the hi and lo A fragments (element e from word e).
// v_perm_b32 picks bytes of the pair {S0, S1} (selector 0-3: S1, 4-7: S0):
// hi dword k = low halves of words 2k, 2k+1; lo dword k = their high halves
__device__ __forceinline__ void frag_hl(const uint32_t (&w)[8], h8& ah, h8& al) {
  u4v h, l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = __builtin_amdgcn_perm(w[2 * k + 1], w[2 * k], 0x05040100u);
    l[k] = __builtin_amdgcn_perm(w[2 * k + 1], w[2 * k], 0x07060302u);
  }
  ah = __builtin_bit_cast(h8, h);
  al = __builtin_bit_cast(h8, l);
}

// the table word at byte offset b (a multiple of 4 below 4N)
__device__ __forceinline__ uint32_t tword(const uint32_t* tb, uint32_t b) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(tb) + b);
}

// B fragments for the four 16-column output tiles of a 32-column block:
// tiles 0, 1 give Re of complex columns 0-15, 16-31, tiles 2, 3 their Im.
// D holds [comp][col][k] halves with comp = (Re hi, Re lo, Im hi, Im lo).
__device__ __forceinline__ void b_frags(const _Float16* D, int ldk, int k, bool part1, int lane, h8 (&bh)[4],
                                        h8 (&bl)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int cc = 16 * (t & 1) + (lane & 15);
    const bool im_tile = t >= 2;
    // re tile: part 0 -> Re, part 1 -> -Im;  im tile: part 0 -> Im, part 1 -> Re
    const int comp = (im_tile != part1) ? 2 : 0;
    const bool neg = part1 && !im_tile;
    const _Float16* ph = D + ((long)comp * 32 + cc) * ldk + k;
    const _Float16* pl = D + ((long)(comp + 1) * 32 + cc) * ldk + k;
    h8 h = *reinterpret_cast<const h8*>(ph);
    h8 l = *reinterpret_cast<const h8*>(pl);
    if (neg) {
      h = -h;
      l = -l;
    }
    bh[t] = h;
    bl[t] = l;
  }
}

__device__ __forceinline__ f4 mma3(const h8& ah, const h8& al, const h8& bh, const h8& bl, f4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------------------
// forward: grid (ceil(nx*r / 32), nc), 256 threads.  Rows u in 16-row tiles,
// tile rt handled by wave rt % 4.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_pdft_fwd(PdftArgs a) {
  constexpr int LDK = N + 8;               // padded k stride of the staged operand
  constexpr int RT_W = (N / 16 + 3) / 4;   // row tiles per wave at most
  constexpr int EPT = N * 32 / 256;        // staged elements per thread
  __shared__ PdftLds<N> L;
  uint32_t* tw0 = L.tw0;
  uint32_t* tw1 = L.tw1;
  _Float16* D = L.D;
  int* s_ky = L.s_ky;
  float* red = L.red;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (halted(a.st, a.check_halt)) return;
  const int nu = a.st->n_units;
  const int c = blockIdx.y, r = a.r, ncols = a.nx * r;
  const int col0 = blockIdx.x * 32;
  load_tables(tw0, tw1, a.tw, N, -1.f);  // part 1: Im of exp(-i theta) = -sin
  for (int u = tid; u < nu; u += 256) s_ky[u] = a.unit_loc[u];
  // V = s_c o U on this block's 32 columns, all y
  float2 v[EPT];
  float amax = 0.f;
  const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * 256, y = e >> 5, cc = e & 31, col = col0 + cc;
    float2 t = make_float2(0.f, 0.f);
    if (col < ncols) t = cmul(coil[(long)y * a.nx + col / r], a.U[(long)y * ncols + col]);
    v[q] = t;
    amax = fmaxf(amax, fmaxf(fabsf(t.x), fabsf(t.y)));
  }
  const float sig = pow2_scale(block_max(amax, red));
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * 256, y = e >> 5, cc = e & 31;
    _Float16 h, l;
    split_hl(v[q].x * sig, h, l);
    D[(0 * 32 + cc) * LDK + y] = h;
    D[(1 * 32 + cc) * LDK + y] = l;
    split_hl(v[q].y * sig, h, l);
    D[(2 * 32 + cc) * LDK + y] = h;
    D[(3 * 32 + cc) * LDK + y] = l;
  }
  __syncthreads();
  const int nrt = (nu + 15) >> 4;
  f4 acc[RT_W][4];
#pragma unroll
  for (int s = 0; s < RT_W; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = f4{0.f, 0.f, 0.f, 0.f};
  // this lane's row of each of its row tiles: ky in bytes of the table
  // (rows past nu take ky = 0; their outputs are not stored, and a row of
  // the product depends on its own A row only)
  uint32_t ky4[RT_W];
#pragma unroll
  for (int s = 0; s < RT_W; ++s) {
    const int u = 16 * (wave + 4 * s) + (lane & 15);
    ky4[s] = (u < nu) ? 4u * (uint32_t)s_ky[u] : 0u;
  }
  auto kloop = [&](const uint32_t* tb, bool part1) {
    for (int y0 = 0; y0 < N; y0 += 32) {
      const int yb = y0 + 8 * (lane >> 4);  // this lane's 8 consecutive y
      h8 bh[4], bl[4];
      b_frags(D, LDK, yb, part1, lane, bh, bl);
#pragma unroll
      for (int s = 0; s < RT_W; ++s) {
        if (wave + 4 * s < nrt) {
          uint32_t w[8];
          uint32_t b = __umul24(ky4[s], (uint32_t)yb);  // 4 ky y, reduced mod 4N per entry
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            w[e] = tword(tb, b & (4u * N - 4u));
            b += ky4[s];
          }
          h8 ah, al;
          frag_hl(w, ah, al);
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[s][t] = mma3(ah, al, bh[t], bl[t], acc[s][t]);
        }
      }
    }
  };
  kloop(tw0, false);
  kloop(tw1, true);
  const float out_scale = a.scale / sig;
  float2* Wc = a.W + (long)c * a.ua * ncols;
#pragma unroll
  for (int s = 0; s < RT_W; ++s) {
    const int rt = wave + 4 * s;
    if (rt < nrt) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = col0 + 16 * t + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = 16 * rt + 4 * (lane >> 4) + q;
          if (u < nu && col < ncols)
            Wc[(long)u * ncols + col] = make_float2(acc[s][t][q] * out_scale, acc[s][t + 2][q] * out_scale);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint + coil combine: grid (ceil(nx*r / 32), coil groups), 256 threads.
// Rows y in 16-row tiles (tile rt on wave rt % 4); per coil the contraction
// runs over the sampled rows u (padded to 32), then conj(s_c) weights the
// result into the group's partial gradient.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_pdft_adj(PdftArgs a) {
  constexpr int LDK = N + 8;
  constexpr int RT_W = (N / 16 + 3) / 4;
  constexpr int EPT = N * 32 / 256;
  __shared__ PdftLds<N> L;
  uint32_t* tw0 = L.tw0;
  uint32_t* tw1 = L.tw1;
  _Float16* D = L.D;
  int* s_ky = L.s_ky;
  float* red = L.red;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (halted(a.st, a.check_halt)) return;
  const int nu = a.st->n_units;
  const int LP = (nu + 31) & ~31;
  const int r = a.r, ncols = a.nx * r;
  const int col0 = blockIdx.x * 32;
  load_tables(tw0, tw1, a.tw, N, 1.f);  // part 1: Im of exp(+i theta) = +sin
  // ky in bytes of the table; rows past nu take ky = 0 (their K rows are zero)
  for (int u = tid; u < N; u += 256) s_ky[u] = (u < nu) ? 4 * a.unit_loc[u] : 0;
  f4 gre[RT_W][2], gim[RT_W][2];
#pragma unroll
  for (int s = 0; s < RT_W; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) gre[s][t] = gim[s][t] = f4{0.f, 0.f, 0.f, 0.f};
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  for (int c = cb; c < ce; ++c) {
    // this coil's K rows on the block's 32 columns; rows past nu are zero
    float2 v[EPT];
    float amax = 0.f;
    const float2* Kc = a.K + (long)c * a.ua * ncols;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * 256, u = e >> 5, cc = e & 31, col = col0 + cc;
      float2 t = make_float2(0.f, 0.f);
      if (u < nu && col < ncols) t = Kc[(long)u * ncols + col];
      v[q] = t;
      amax = fmaxf(amax, fmaxf(fabsf(t.x), fabsf(t.y)));
    }
    const float sig = pow2_scale(block_max(amax, red));  // its barriers also retire the previous coil's reads
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * 256, u = e >> 5, cc = e & 31;
      _Float16 h, l;
      split_hl(v[q].x * sig, h, l);
      D[(0 * 32 + cc) * LDK + u] = h;
      D[(1 * 32 + cc) * LDK + u] = l;
      split_hl(v[q].y * sig, h, l);
      D[(2 * 32 + cc) * LDK + u] = h;
      D[(3 * 32 + cc) * LDK + u] = l;
    }
    __syncthreads();
    f4 acc[RT_W][4];
#pragma unroll
    for (int s = 0; s < RT_W; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[s][t] = f4{0.f, 0.f, 0.f, 0.f};
    auto kloop = [&](const uint32_t* tb, bool part1) {
      for (int u0 = 0; u0 < LP; u0 += 32) {
        const int ub = u0 + 8 * (lane >> 4);  // this lane's 8 consecutive u
        h8 bh[4], bl[4];
        b_frags(D, LDK, ub, part1, lane, bh, bl);
        const int4 ka = *reinterpret_cast<const int4*>(s_ky + ub);
        const int4 kb = *reinterpret_cast<const int4*>(s_ky + ub + 4);
        const uint32_t k4[8] = {(uint32_t)ka.x, (uint32_t)ka.y, (uint32_t)ka.z, (uint32_t)ka.w,
                                (uint32_t)kb.x, (uint32_t)kb.y, (uint32_t)kb.z, (uint32_t)kb.w};
        // 4 ky y for this lane's row of row tile s: y = y0 + 64 s
        // (the increments are hidden from the optimiser, which would
        // otherwise fold the sums back into a 32-bit multiply per tile)
        const uint32_t y0 = 16 * wave + (lane & 15);
        uint32_t pk[8], inc[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          pk[e] = k4[e] * y0;
          inc[e] = k4[e] << 6;
          asm volatile("" : "+v"(inc[e]));
        }
#pragma unroll
        for (int s = 0; s < RT_W; ++s) {
          if (s > 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) pk[e] += inc[e];
          }
          if (16 * (wave + 4 * s) < N) {
            uint32_t w[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = tword(tb, pk[e] & (4u * N - 4u));
            h8 ah, al;
            frag_hl(w, ah, al);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[s][t] = mma3(ah, al, bh[t], bl[t], acc[s][t]);
          }
        }
      }
    };
    kloop(tw0, false);
    kloop(tw1, true);
    // conj(s_c) o T_c into the partial gradient
    const float inv = 1.f / sig;
    const float2* coil = a.coils + (long)c * a.n;
#pragma unroll
    for (int s = 0; s < RT_W; ++s) {
      const int rt = wave + 4 * s;
      if (16 * rt < N) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int col = col0 + 16 * t + (lane & 15);
          const int x = (col < ncols) ? col / r : 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int y = 16 * rt + 4 * (lane >> 4) + q;
            const float2 sc = coil[(long)y * a.nx + x];
            const float tr = acc[s][t][q] * inv, ti = acc[s][t + 2][q] * inv;
            gre[s][t][q] += sc.x * tr + sc.y * ti;
            gim[s][t][q] += sc.x * ti - sc.y * tr;
          }
        }
      }
    }
  }
  float2* out = a.G + (long)blockIdx.y * a.part_stride;
#pragma unroll
  for (int s = 0; s < RT_W; ++s) {
    const int rt = wave + 4 * s;
    if (16 * rt < N) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = col0 + 16 * t + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int y = 16 * rt + 4 * (lane >> 4) + q;
          if (col < ncols) out[(long)y * ncols + col] = make_float2(gre[s][t][q] * a.scale, gim[s][t][q] * a.scale);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// N = 256 factored as 16 x 16: the same transforms as two dense 16-point DFT
// stages on the matrix cores with a twiddle between them (w_m = exp(-2 pi i / m)):
//   forward  (y = 16 y1 + y2, ky = k1 + 16 k2)
//     A[k1][y2] = w256^(k1 y2) sum_y1 w16^(k1 y1) V[16 y1 + y2],
//     W[k1 + 16 k2] = sum_y2 w16^(k2 y2) A[k1][y2];
//   adjoint  (ky = k1 + 16 k2, y = y1 + 16 y2, conjugate exponents)
//     B[k1][y1] = w256^(-k1 y1) sum_k2 w16^(-k2 y1) K[k1 + 16 k2],
//     T[y1 + 16 y2] = sum_k1 w16^(-k1 y2) B[k1][y1].
// Each stage multiplies the fixed 16-point DFT matrix F = C -+ i S (the A
// operand: [C | +-S] for real outputs against B = [Re; Im], [C | -+S] for
// imaginary outputs against [Im; Re], its fp16 hi and lo halves in registers)
// by 16 complex data columns (the B operand).  The data are staged in LDS as
// fp16 hi and lo planes [comp][hl][n][kappa] (the 16 contraction values of
// a column n contiguous: one 16-byte read per fragment) after a power-of-two
// scale that keeps every stage input within 2^14 (inputs at most 2^10; a
// 16-point stage grows a magnitude at most 16 times).  Products keep
// hi*hi + hi*lo + lo*hi with FP32 accumulation.  A workgroup of 4 waves
// takes 16 columns col = x*r + j (the data columns n of every product) and a
// group of coils; in each stage wave w takes the batches w, w+4, w+8, w+12.
// ---------------------------------------------------------------------------
// the A fragments of F (sgn = +1 forward, -1 inverse): lane l holds row
// m = l%16, contraction entries kappa = 8(l/16) + e (kappa < 16: C[m][kappa],
// else the signed S[m][kappa - 16])
__device__ __forceinline__ void dft16_frags(const float2* tw256, float sgn, int lane, h8& re_h, h8& re_l, h8& im_h,
                                            h8& im_l) {
  const int m = lane & 15, kb = 8 * (lane >> 4);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int kap = kb + e, k = kap & 15;
    const float2 w = tw256[16 * ((m * k) & 15)];  // exp(-2 pi i m k / 16) = (C, -S)
    const float cv = w.x, sv = -w.y;
    const float vre = kap < 16 ? cv : sgn * sv;
    const float vim = kap < 16 ? cv : -sgn * sv;
    _Float16 h, l;
    split_hl(vre, h, l);
    re_h[e] = h;
    re_l[e] = l;
    split_hl(vim, h, l);
    im_h[e] = h;
    im_l[e] = l;
  }
}

// plane geometry (halves): a row n holds the 16 contraction values, padded to
// PR so that the four row groups of a wave's scattered writes fall in
// different LDS banks; planes (Re hi, Re lo, Im hi, Im lo) follow each other
template <int PR_>
struct Planes {
  static constexpr int PR = PR_, PP = 16 * PR_, PCOL = 4 * PP + 8;  // row, plane, column (padded) strides
};
using P1 = Planes<16>;  // staged inputs: whole rows written at once, the column stride padded
using P2g = Planes<24>; // stage-2 inputs: scattered row writes, the row stride padded

// one stage on the column whose planes start at P: D_re, D_im[v] of lane l
// hold output row 4(l/16)+v, column l%16
template <typename G>
__device__ __forceinline__ void dft16_stage(const _Float16* P, int lane, const h8& re_h, const h8& re_l,
                                            const h8& im_h, const h8& im_l, f4& d_re, f4& d_im) {
  constexpr int PR = G::PR, PP = G::PP;
  const int comp = lane >> 5, n = lane & 15, kb = 8 * ((lane >> 4) & 1);
  const _Float16* pre = P + comp * 2 * PP + n * PR + kb;        // B_re = [Re; Im]
  const _Float16* pim = P + (1 - comp) * 2 * PP + n * PR + kb;  // B_im = [Im; Re]
  const h8 brh = *reinterpret_cast<const h8*>(pre), brl = *reinterpret_cast<const h8*>(pre + PP);
  const h8 bih = *reinterpret_cast<const h8*>(pim), bil = *reinterpret_cast<const h8*>(pim + PP);
  d_re = mma3(re_h, re_l, brh, brl, f4{0.f, 0.f, 0.f, 0.f});
  d_im = mma3(im_h, im_l, bih, bil, f4{0.f, 0.f, 0.f, 0.f});
}

// four consecutive contraction values k0..k0+3 of row n into the four planes
// (one 8-byte write per plane; k0 a multiple of 4)
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void put_hl4(_Float16* P, int n, int k0, const float2 (&z)[4]) {
  constexpr int PR = P2g::PR, PP = P2g::PP;
  h4 rh, rl, ih, il;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    _Float16 h, l;
    split_hl(z[q].x, h, l);
    rh[q] = h;
    rl[q] = l;
    split_hl(z[q].y, h, l);
    ih[q] = h;
    il[q] = l;
  }
  const int o = n * PR + k0;
  *reinterpret_cast<h4*>(P + o) = rh;
  *reinterpret_cast<h4*>(P + PP + o) = rl;
  *reinterpret_cast<h4*>(P + 2 * PP + o) = ih;
  *reinterpret_cast<h4*>(P + 3 * PP + o) = il;
}

// 16 contiguous values of one column (kappa = 0..15) into the four planes at row n
__device__ __forceinline__ void put_row16(_Float16* P, int n, const float2 (&v)[16], float sig) {
  constexpr int PR = P1::PR, PP = P1::PP;
  h8 rh[2], rl[2], ih[2], il[2];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    _Float16 h, l;
    split_hl(v[k].x * sig, h, l);
    rh[k >> 3][k & 7] = h;
    rl[k >> 3][k & 7] = l;
    split_hl(v[k].y * sig, h, l);
    ih[k >> 3][k & 7] = h;
    il[k >> 3][k & 7] = l;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    *reinterpret_cast<h8*>(P + n * PR + 8 * b) = rh[b];
    *reinterpret_cast<h8*>(P + PP + n * PR + 8 * b) = rl[b];
    *reinterpret_cast<h8*>(P + 2 * PP + n * PR + 8 * b) = ih[b];
    *reinterpret_cast<h8*>(P + 3 * PP + n * PR + 8 * b) = il[b];
  }
}

// The data of one stage: 16 sets (the batch index of the stage: y2 or k1 in
// stage 1, k1 or y1 in stage 2), each 16 data columns n = the workgroup's
// columns.  Stage 1 reads its sets from the staged inputs; its outputs go
// to registers, then (after a barrier) into the stage-2 sets in the same
// LDS buffer; stage 2 writes whole runs of the 16 columns per output row.
constexpr int S1 = P1::PCOL;  // stage-1 set stride (halves)
constexpr int S2 = P2g::PCOL; // stage-2 set stride: 4 sets apart land 64 bytes apart in the banks
constexpr int PDFT16_LDS = 16 * (S1 > S2 ? S1 : S2);

// forward: grid (ceil(nx r / 16), coil groups), 256 threads
__global__ __launch_bounds__(256) void k_pdft16_fwd(PdftArgs a) {
  constexpr int N = 256;
  __shared__ float2 s_tw[N];
  __shared__ int s_ro[N];  // ky -> its row u of W, -1 if not sampled
  __shared__ float red[4];
  __shared__ __attribute__((aligned(16))) _Float16 D[PDFT16_LDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = a.r, ncols = a.nx * r, col0 = blockIdx.x * 16;
  // staging: this thread's column and y2 (rows y = 16 y1 + y2 of U), requested first
  const int cl = tid & 15, y2t = tid >> 4, col = col0 + cl;
  const bool cok = col < ncols;
  const int colc = cok ? col : 0, x = colc / r;
  float2 uv[16];
#pragma unroll
  for (int y1 = 0; y1 < 16; ++y1) uv[y1] = a.U[(long)(16 * y1 + y2t) * ncols + colc];
  s_tw[tid] = a.tw[tid];
  s_ro[tid] = -1;
  if (halted(a.st, a.check_halt)) return;
  const int nu = a.st->n_units;
  __syncthreads();
  for (int u = tid; u < nu; u += 256) s_ro[a.unit_loc[u]] = u;
  __syncthreads();
  h8 fre_h, fre_l, fim_h, fim_l;
  dft16_frags(s_tw, 1.f, lane, fre_h, fre_l, fim_h, fim_l);
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  const int n = lane & 15, g4 = 4 * (lane >> 4);
  const bool ook = col0 + n < ncols;  // this lane's output column
  for (int c = cb; c < ce; ++c) {
    // V = s_c o U on this thread's 16 rows: set y2, row cl
    // (every load issued from a valid address, then masked: a load under a
    // branch would wait alone)
    const float2* coil = a.coils + (long)c * a.n + x;
    float2 v[16];
#pragma unroll
    for (int y1 = 0; y1 < 16; ++y1) v[y1] = coil[(long)(16 * y1 + y2t) * a.nx];
    float amax = 0.f;
#pragma unroll
    for (int y1 = 0; y1 < 16; ++y1) {
      v[y1] = cok ? cmul(v[y1], uv[y1]) : make_float2(0.f, 0.f);
      amax = fmaxf(amax, fmaxf(fabsf(v[y1].x), fabsf(v[y1].y)));
    }
    // its barriers also retire the previous coil's reads of D
    const float sig = pow2_scale(block_max(amax, red)) * (1.f / 16.f);
    put_row16(D + y2t * S1, cl, v, sig);
    __syncthreads();
    // stage 1 on sets y2 = 4 wave + q: rows k1 = 4(l/16)+v, then w256^(k1 y2)
    float2 z[4][4];  // [v][q]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y2 = 4 * wave + q;
      f4 dre, dim;
      dft16_stage<P1>(D + y2 * S1, lane, fre_h, fre_l, fim_h, fim_l, dre, dim);
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) z[vv][q] = cmul(make_float2(dre[vv], dim[vv]), s_tw[((g4 + vv) * y2) & 255]);
    }
    __syncthreads();
    // stage-2 sets k1: row n (column), contraction y2 (this wave's four at once)
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) put_hl4(D + (g4 + vv) * S2, n, 4 * wave, z[vv]);
    __syncthreads();
    // stage 2 on sets k1 = wave + 4q: rows k2 = 4(l/16)+v, ky = k1 + 16 k2
    const float os = a.scale / sig;
    float2* Wc = a.W + (long)c * a.ua * ncols + col0 + n;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k1 = wave + 4 * q;
      f4 dre, dim;
      dft16_stage<P2g>(D + k1 * S2, lane, fre_h, fre_l, fim_h, fim_l, dre, dim);
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int u = s_ro[k1 + 16 * (g4 + vv)];
        if (u >= 0 && ook) Wc[(long)u * ncols] = make_float2(dre[vv] * os, dim[vv] * os);
      }
    }
  }
}

// adjoint + coil combine: grid (ceil(nx r / 16), coil groups), 256 threads;
// group g writes its partial gradient to G + g part_stride
__global__ __launch_bounds__(256) void k_pdft16_adj(PdftArgs a) {
  constexpr int N = 256;
  __shared__ float2 s_tw[N];
  __shared__ int s_ro[N];
  __shared__ float red[4];
  __shared__ __attribute__((aligned(16))) _Float16 D[PDFT16_LDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = a.r, ncols = a.nx * r, col0 = blockIdx.x * 16;
  const int cl = tid & 15, k1t = tid >> 4, col = col0 + cl;
  const bool cok = col < ncols;
  const int colc = cok ? col : 0;
  s_tw[tid] = a.tw[tid];
  s_ro[tid] = -1;
  if (halted(a.st, a.check_halt)) return;
  const int nu = a.st->n_units;
  __syncthreads();
  for (int u = tid; u < nu; u += 256) s_ro[a.unit_loc[u]] = u;
  __syncthreads();
  h8 fre_h, fre_l, fim_h, fim_l;
  dft16_frags(s_tw, -1.f, lane, fre_h, fre_l, fim_h, fim_l);
  const int n = lane & 15, g4 = 4 * (lane >> 4);
  const bool ook = col0 + n < ncols;
  const int xo = min(col0 + n, ncols - 1) / r;  // this lane's output column's image column
  float2 acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) acc[q][vv] = make_float2(0.f, 0.f);
  const int cb = blockIdx.y * a.cgs, ce = min(a.nc, cb + a.cgs);
  for (int c = cb; c < ce; ++c) {
    // this thread's 16 rows ky = k1 + 16 k2 of K (zero where not sampled): set k1, row cl
    // (loads from valid addresses, then masked)
    const float2* Kc = a.K + (long)c * a.ua * ncols + colc;
    float2 v[16];
    bool ok[16];
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      const int u = s_ro[k1t + 16 * k2];
      ok[k2] = cok && u >= 0;
      v[k2] = Kc[(long)max(u, 0) * ncols];
    }
    float amax = 0.f;
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      if (!ok[k2]) v[k2] = make_float2(0.f, 0.f);
      amax = fmaxf(amax, fmaxf(fabsf(v[k2].x), fabsf(v[k2].y)));
    }
    // this lane's coil values at its outputs y = y1 + 16 y2 (y1 = wave + 4q, y2 = 4(l/16)+v)
    const float2* coil = a.coils + (long)c * a.n + xo;
    float2 cw[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) cw[q][vv] = coil[(long)(wave + 4 * q + 16 * (g4 + vv)) * a.nx];
    const float sig = pow2_scale(block_max(amax, red)) * (1.f / 16.f);
    put_row16(D + k1t * S1, cl, v, sig);
    __syncthreads();
    // stage 1 on sets k1 = 4 wave + q: rows y1 = 4(l/16)+v, then w256^(-k1 y1)
    float2 z[4][4];  // [v][q]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k1 = 4 * wave + q;
      f4 dre, dim;
      dft16_stage<P1>(D + k1 * S1, lane, fre_h, fre_l, fim_h, fim_l, dre, dim);
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const float2 w = s_tw[((g4 + vv) * k1) & 255];
        z[vv][q] = cmul(make_float2(dre[vv], dim[vv]), make_float2(w.x, -w.y));
      }
    }
    __syncthreads();
    // stage-2 sets y1: row n (column), contraction k1 (this wave's four at once)
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) put_hl4(D + (g4 + vv) * S2, n, 4 * wave, z[vv]);
    __syncthreads();
    // stage 2 on sets y1 = wave + 4q: rows y2 = 4(l/16)+v; conj(s_c) weighting
    const float inv = 1.f / sig;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y1 = wave + 4 * q;
      f4 dre, dim;
      dft16_stage<P2g>(D + y1 * S2, lane, fre_h, fre_l, fim_h, fim_l, dre, dim);
#pragma unroll
      for (int vv = 0; vv < 4; ++vv)
        acc[q][vv] = cjfma(acc[q][vv], cw[q][vv], make_float2(dre[vv] * inv, dim[vv] * inv));
    }
  }
  if (ook) {
    float2* out = a.G + (long)blockIdx.y * a.part_stride + col0 + n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv)
        out[(long)(wave + 4 * q + 16 * (g4 + vv)) * ncols] = cscale(acc[q][vv], a.scale);
  }
}

hipError_t launch_pdft(int which, int ny, const PdftArgs& a, int grid_x, int grid_y, hipStream_t s) {
  const dim3 g(grid_x, grid_y), b(256);
#define AG_PDFT(NN)                                                      \
  case NN:                                                               \
    if (which == 0) hipLaunchKernelGGL(k_pdft_fwd<NN>, g, b, 0, s, a);   \
    else hipLaunchKernelGGL(k_pdft_adj<NN>, g, b, 0, s, a);              \
    break;
  if (ny == 256) {  // the factored form: 16 columns per workgroup
    const dim3 g16((a.nx * a.r + 15) / 16, grid_y);
    if (which == 0) hipLaunchKernelGGL(k_pdft16_fwd, g16, b, 0, s, a);
    else hipLaunchKernelGGL(k_pdft16_adj, g16, b, 0, s, a);
    return hipGetLastError();
  }
  switch (ny) {
    AG_PDFT(32)
    AG_PDFT(64)
    AG_PDFT(128)
    AG_PDFT(256)
    default:
      return hipErrorInvalidValue;
  }
#undef AG_PDFT
  return hipGetLastError();
}

}  // namespace ag
