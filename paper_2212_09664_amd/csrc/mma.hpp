// The 16x16x4 matrix-core tiles shared by the Gram kernels: FP32 and FP64
// accumulators, their lane layout and the reductions of per-wave tiles.
#pragma once

#include "kernels_core.hpp"

namespace ag {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
  using V = f4v;
  __device__ static V zero() { return V{0.f, 0.f, 0.f, 0.f}; }
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // accumulator register v of lane l holds D[row(l, v)][l % 16]
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mma<double> {
  using V = d4v;
  __device__ static V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// Lane layout of the 16x16x4 MFMA (both types): lane l holds A[l%16][l/16] and
// B[l/16][l%16].  The accumulator differs: register v of lane l holds
// D[4*(l/16) + v][l%16] for f32 and D[4*v + l/16][l%16] for f64.

// Sum the NW waves' tile (one 16x16 accumulator per wave) into LDS buffer t.
template <typename T, int NW>
__device__ __forceinline__ void tile_reduce_n(T* t, const typename Mma<T>::V& acc, int wave, int lane) {
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int idx = Mma<T>::row(lane, v) * 16 + (lane & 15);
        t[idx] = (w == 0) ? acc[v] : t[idx] + acc[v];
      }
    }
    __syncthreads();
  }
}

// Sum NTL tiles over the NW waves (one 16x16 accumulator per tile and wave)
// into out[tile * 256 + entry] with two barriers: every wave writes its tiles
// to scratch (NW * NTL * 256 values), then the workgroup adds them up in
// wave order (the order of tile_reduce_n, so the sums are the same).
template <typename T, int NW, int NTL>
__device__ __forceinline__ void tiles_reduce_par(T* out, T* scratch, const typename Mma<T>::V (&acc)[NTL], int wave,
                                                 int lane) {
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) scratch[(wave * NTL + t) * 256 + Mma<T>::row(lane, v) * 16 + (lane & 15)] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < NTL * 256; e += blockDim.x) {
    T sum = scratch[e];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += scratch[w * NTL * 256 + e];
    out[e] = sum;
  }
  __syncthreads();
}

}  // namespace ag
