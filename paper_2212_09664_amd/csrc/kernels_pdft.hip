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

hipError_t launch_pdft(int which, int ny, const PdftArgs& a, int grid_x, int grid_y, hipStream_t s) {
  const dim3 g(grid_x, grid_y), b(256);
#define AG_PDFT(NN)                                                      \
  case NN:                                                               \
    if (which == 0) hipLaunchKernelGGL(k_pdft_fwd<NN>, g, b, 0, s, a);   \
    else hipLaunchKernelGGL(k_pdft_adj<NN>, g, b, 0, s, a);              \
    break;
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
