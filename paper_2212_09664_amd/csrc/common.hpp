// Shared device helpers for the altGDmin kernels (gfx950): complex
// arithmetic, the device-side state block and an LDS-staged Stockham FFT.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AG_NT 256  // threads per workgroup for the streaming kernels

// ---------------------------------------------------------------------------
// complex helpers (interleaved float2 / double2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cjmul(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulj(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
// acc + a * b and acc + a * conj(b) as two fused multiply-adds per part
// (cadd(acc, cmul(a, b)) costs six instructions: the sum is rounded apart)
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(-a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(a.y, b.x, fmaf(a.x, b.y, acc.y)));
}
__device__ __forceinline__ float2 cfmaj(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(-a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// acc + conj(a) * b
__device__ __forceinline__ float2 cjfma(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(-a.y, b.x, fmaf(a.x, b.y, acc.y)));
}

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 djmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 f2d(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ float2 d2f(double2 a) { return make_float2((float)a.x, (float)a.y); }

// ---------------------------------------------------------------------------
// device state (one block at the start of the workspace)
// ---------------------------------------------------------------------------
struct DevState {
  int32_t err;        // 0 or an altgdmin_status
  int32_t err_frame;  // frame of a non-positive-definite Gram, -1 otherwise
  int32_t halt;       // 1: every later kernel of the loop returns at once
  int32_t step_ok;    // 1: the current iteration's GD + QR step is applied
  int32_t t;          // iterations completed
  int32_t exited;     // exit rule fired
  int32_t converged;  // stationary start (grad_0 = 0)
  int32_t n_units;    // distinct sampled lines (LINES) / locations (INDEX)
  double eta;         // step size (<= 0: not yet set)
  double gamma;       // truncation threshold
  double ysq;         // sum_k ||y_k||^2
  double mbar;        // mean samples per coil
  double f;           // cost of the last iteration
  double sd;          // SD(U_{t-1}, U_t)
  double grad_norm;   // ||grad||_F of the last iteration
  double cost_out;    // scratch for altgdmin_cost
  int32_t n_gwork;    // LINES: (line, sample tile) work items of the Gram kernel
  int32_t step_flags; // the fused QR step's outcome, committed after it (STEP_*)
  double eta_next;    // the step size it used (committed after it)
  int32_t stats_pending;  // 1: f, sd and grad_norm of the last step wait in the statistics inputs
  int32_t n_trunc;    // samples zeroed by the truncation of the last initialisation
  int32_t exit_run;   // consecutive iterations that met the exit test
  int32_t pad_e;
  double pad[2];
};
// the loop's stop test: err and halt both requested before either is tested
// (a short-circuit test waits for one load before issuing the other)
__device__ __forceinline__ bool halted(const DevState* st, int check_halt) {
  const int e = st->err, h = st->halt;
  return (e | (h & -(check_halt != 0))) != 0;
}
#define STEP_APPLIED 1
#define STEP_EXIT 2
#define STEP_CONVERGED 4

// ---------------------------------------------------------------------------
// in-register DFTs of radix 2, 4, 8, 16
// Output k of the radix-R DFT ends up in register out_pos<R>(k).
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 v) {  // * (-i) forward, * (+i) inverse
  return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = csub(a1, a3);
  float2 t = mul_mi<INV>(d13);
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, t);
  a3 = csub(d02, t);
}

// v * exp(-+ 2 pi i k / 16), k a compile-time constant after unrolling
template <bool INV>
__device__ __forceinline__ float2 tw16(float2 v, int k) {
  const float C1 = 0.92387953251128674f, C2 = 0.70710678118654752f, C3 = 0.38268343236508977f;
  float c, s;
  switch (k & 15) {
    case 0: return v;
    case 1: c = C1; s = C3; break;
    case 2: c = C2; s = C2; break;
    case 3: c = C3; s = C1; break;
    case 4: return mul_mi<INV>(v);
    case 5: c = -C3; s = C1; break;
    case 6: c = -C2; s = C2; break;
    case 7: c = -C1; s = C3; break;
    case 8: return make_float2(-v.x, -v.y);
    case 9: c = -C1; s = -C3; break;
    default: c = 1.f; s = 0.f; break;
  }
  // forward: (c - i s); inverse: (c + i s)
  float2 w = INV ? make_float2(c, s) : make_float2(c, -s);
  return cmul(v, w);
}

template <int R>
__device__ __forceinline__ constexpr int out_pos(int k) {
  return R == 16 ? 4 * (k % 4) + k / 4 : (R == 8 ? 4 * (k % 2) + k / 2 : k);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* v) {
  if constexpr (R == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // n = 4a + b, k = c + 2d
#pragma unroll
    for (int b = 0; b < 4; ++b) dft2<INV>(v[b], v[4 + b]);
#pragma unroll
    for (int b = 1; b < 4; ++b) v[4 + b] = tw16<INV>(v[4 + b], 2 * b);
#pragma unroll
    for (int c = 0; c < 2; ++c) dft4<INV>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  } else if constexpr (R == 16) {
    // n = 4a + b, k = c + 4d
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4<INV>(v[b], v[4 + b], v[8 + b], v[12 + b]);
#pragma unroll
    for (int c = 1; c < 4; ++c)
#pragma unroll
      for (int b = 1; b < 4; ++b) v[4 * c + b] = tw16<INV>(v[4 * c + b], b * c);
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4<INV>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  }
}

// ---------------------------------------------------------------------------
// Stockham autosort FFT of TX columns of length N held in LDS as s[e*TX+col]
// (column index fastest), by NT threads (thread index modulo NT: a
// workgroup of several groups of NT threads transforms one tile per group,
// every group reaching the barriers together).  Each pass of radix R reads R points at stride
// N/R, applies the twiddles exp(-+2 pi i (j mod Ns) r / (Ns R)), does an
// in-register radix-R DFT and writes them at stride Ns.  tw[t] holds
// exp(-2 pi i t / N) in float (computed in double).  Unnormalised.
// ---------------------------------------------------------------------------
template <int N, int R, int TX, int NT, bool INV, bool CONJ_TW = INV>
__device__ __forceinline__ void stockham_pass(float2* s, const float2* __restrict__ tw, int Ns) {
  constexpr int G = TX * (N / R);
  constexpr int IT = (G + NT - 1) / NT;
  float2 v[IT][R];
  const int tid = threadIdx.x % NT;  // a workgroup of several NT-thread groups runs one transform per group
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * NT;
    if ((G % NT == 0) || g < G) {
      const int col = g % TX, j = g / TX;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = s[(j + r * (N / R)) * TX + col];
      if (Ns > 1) {
        const int step = (j % Ns) * (N / (Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[step * r];
          if (CONJ_TW) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      dft_reg<R, INV>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * NT;
    if ((G % NT == 0) || g < G) {
      const int col = g % TX, j = g / TX;
      const int idxD = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) s[(idxD + r * Ns) * TX + col] = v[it][out_pos<R>(r)];
    }
  }
  __syncthreads();
}

// The whole transform; N a power of two in [8, 512].
template <int N, int TX, int NT, bool INV>
__device__ __forceinline__ void fft_lds(float2* s, const float2* __restrict__ tw) {
  if constexpr (N == 8) {
    stockham_pass<8, 8, TX, NT, INV>(s, tw, 1);
  } else if constexpr (N == 16) {
    stockham_pass<16, 16, TX, NT, INV>(s, tw, 1);
  } else if constexpr (N == 32) {
    stockham_pass<32, 8, TX, NT, INV>(s, tw, 1);
    stockham_pass<32, 4, TX, NT, INV>(s, tw, 8);
  } else if constexpr (N == 64) {
    stockham_pass<64, 8, TX, NT, INV>(s, tw, 1);
    stockham_pass<64, 8, TX, NT, INV>(s, tw, 8);
  } else if constexpr (N == 128) {
    stockham_pass<128, 16, TX, NT, INV>(s, tw, 1);
    stockham_pass<128, 8, TX, NT, INV>(s, tw, 16);
  } else if constexpr (N == 256) {
    stockham_pass<256, 16, TX, NT, INV>(s, tw, 1);
    stockham_pass<256, 16, TX, NT, INV>(s, tw, 16);
  } else if constexpr (N == 512) {
    stockham_pass<512, 8, TX, NT, INV>(s, tw, 1);
    stockham_pass<512, 8, TX, NT, INV>(s, tw, 8);
    stockham_pass<512, 8, TX, NT, INV>(s, tw, 64);
  }
}

// ---------------------------------------------------------------------------
// The same transform with its first pass fed from registers and its last
// pass left in registers: only the passes in between go through LDS.
//   input  item (it, r) of thread t, g = t + it*NT: row g/TX + r*(N/R0),
//          column g%TX;
//   output item (it, r): row out_row(g, r), column g%TX.
// tw[t] = exp(-+2 pi i t / N) in the transform's own direction (the caller
// passes the conjugated table for the inverse).  For N <= 16 (one pass) no
// LDS is touched.  The function returns with the LDS tile free for reuse
// (its last LDS read is followed by a barrier).
// ---------------------------------------------------------------------------
template <int N> struct FftPlan;
template <> struct FftPlan<8>   { static constexpr int P = 1, R0 = 8,  RL = 8;  };
template <> struct FftPlan<16>  { static constexpr int P = 1, R0 = 16, RL = 16; };
template <> struct FftPlan<32>  { static constexpr int P = 2, R0 = 8,  RL = 4;  };
template <> struct FftPlan<64>  { static constexpr int P = 2, R0 = 8,  RL = 8;  };
template <> struct FftPlan<128> { static constexpr int P = 2, R0 = 16, RL = 8;  };
template <> struct FftPlan<256> { static constexpr int P = 2, R0 = 16, RL = 16; };
template <> struct FftPlan<512> { static constexpr int P = 3, R0 = 8,  RL = 8;  };

template <int N, int TX, int NT>
struct FftGeom {
  using PL = FftPlan<N>;
  static constexpr int R0 = PL::R0, RL = PL::RL;
  static constexpr int G0 = TX * (N / R0), IT0 = (G0 + NT - 1) / NT;
  static constexpr int GL = TX * (N / RL), ITL = (GL + NT - 1) / NT;
  __device__ static bool in_ok(int g) { return (G0 % NT == 0) || g < G0; }
  __device__ static bool out_ok(int g) { return (GL % NT == 0) || g < GL; }
  __device__ static int in_row(int g, int r) { return g / TX + r * (N / R0); }
  __device__ static int out_row(int g, int r) {
    return PL::P == 1 ? (g / TX) * R0 + r : g / TX + r * (N / RL);
  }
};

template <int N, int TX, int NT, bool INV, int IT0_, int R0_, int ITL_, int RL_>
__device__ __forceinline__ void fft_regs(float2 (&v0)[IT0_][R0_], float2 (&vo)[ITL_][RL_], float2* s,
                                         const float2* __restrict__ tw) {
  using GM = FftGeom<N, TX, NT>;
  static_assert(IT0_ == GM::IT0 && R0_ == GM::R0 && ITL_ == GM::ITL && RL_ == GM::RL,
                "register tiles do not match the plan");
  constexpr int R0 = GM::R0, RL = GM::RL, P = FftPlan<N>::P;
  const int tid = threadIdx.x % NT;
#pragma unroll
  for (int it = 0; it < GM::IT0; ++it)
    if (GM::in_ok(tid + it * NT)) dft_reg<R0, INV>(v0[it]);
  if constexpr (P == 1) {
#pragma unroll
    for (int it = 0; it < GM::IT0; ++it)
#pragma unroll
      for (int r = 0; r < R0; ++r) vo[it][r] = v0[it][out_pos<R0>(r)];
    return;
  } else {
    // first pass: Ns = 1, outputs to rows j*R0 + r
#pragma unroll
    for (int it = 0; it < GM::IT0; ++it) {
      const int g = tid + it * NT;
      if (GM::in_ok(g)) {
        const int col = g % TX, j = g / TX;
#pragma unroll
        for (int r = 0; r < R0; ++r) s[(j * R0 + r) * TX + col] = v0[it][out_pos<R0>(r)];
      }
    }
    __syncthreads();
    if constexpr (P == 3) stockham_pass<N, 8, TX, NT, INV, false>(s, tw, R0);
    // last pass: Ns = N/RL, reads rows j + r*Ns, outputs rows j + r*Ns
#pragma unroll
    for (int it = 0; it < GM::ITL; ++it) {
      const int g = tid + it * NT;
      if (GM::out_ok(g)) {
        const int col = g % TX, j = g / TX;
#pragma unroll
        for (int r = 0; r < RL; ++r) vo[it][r] = s[(j + r * (N / RL)) * TX + col];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < GM::ITL; ++it) {
      const int g = tid + it * NT;
      if (GM::out_ok(g)) {
        const int j = g / TX;
#pragma unroll
        for (int r = 1; r < RL; ++r) vo[it][r] = cmul(vo[it][r], tw[j * r]);
        dft_reg<RL, INV>(vo[it]);
        float2 t[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) t[r] = vo[it][out_pos<RL>(r)];
#pragma unroll
        for (int r = 0; r < RL; ++r) vo[it][r] = t[r];
      }
    }
  }
}

// Columns per workgroup for a transform of length N: keeps the LDS tile at
// N*TX*8 bytes <= 32 KB with TX in [4, 32].
template <int N>
struct ColTile {
  static constexpr int TX = (N >= 512) ? 8 : (N >= 256 ? 16 : (N >= 128 ? 32 : 32));
};
