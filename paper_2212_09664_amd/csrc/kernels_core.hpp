// Argument blocks and launchers of the non-transform kernels.
#pragma once

#include "kernels.hpp"

#define GRAM_OPT 2    // outputs per thread in the per-line Gram kernels
#define SOLVE_NT 1024  // threads of the per-frame solve
#define QR_NSM 2       // QR Gram: streams of 4 waves per workgroup
#define GRAM_NWG 1     // per-line Gram: groups of 4 waves per workgroup
#define GRAM_INDEX_CHUNK 512  // general masks: samples per Gram workgroup (one coil)
#define GRAM_DS32 2    // per-line Gram, FP32: steps whose loads are issued together
#define GRAM_DS64 4    // the same for FP64
#define GCOLS_OPT 9   // outputs per thread in the column-Gram kernel (m <= 128)
#define GCOLS_NT 1024

namespace ag {

// one complex Jacobi rotation: c, s and the phase e = exp(-i phi)
struct JRot {
  double c, s;
  double2 e;
};

struct JacobiScratch {
  double red[1024];
  JRot rot[64];     // this round's rotations, one per pair
  int2 pq[64];      // and their index pairs
  int top[128];     // per index: among the r_top largest diagonal entries
  double bnd[128];  // per index: Gershgorin bound within its block
};

struct GramLinesArgs {
  const float2* W;       // [c][u][x][j], ua rows per coil
  const float2* yu;      // per-line data [c][p][x]
  const float2* yg;      // per work item: [c][x][8 samples]
  const int4* items;     // work items (line, sample tile of 8, first pair, pair count)
  const int2* pairs;
  const int32_t* loc_ptr;
  const int32_t* unit_loc;
  int nc, r, nx, ua;
  int cg;                // coils per workgroup (coil group)
  long npairs;           // allocated pairs per group in hp
  double2* P;            // [g][u][r][r]
  double2* hp;           // [g][pair][r]
  DevState* st;
  int check_halt;
};

struct GramIndexArgs {
  const float2* W;       // [c][loc][j]
  const float2* y;       // [k][c][m_max]
  const int32_t* mask;
  const int32_t* m_k;
  int nc, r, n, m_max;
  int chunk;             // samples per workgroup
  int nchunks;           // chunks per frame
  double2* part;         // [k][chunk][c][r*r + r]
  DevState* st;
  int check_halt;
};

struct SolveArgs {
  const double2* P;      // LINES: per-line Grams; INDEX: chunk partials
  const double2* hp;
  const int32_t* mask;
  const int32_t* m_k;
  const int32_t* pair_of;
  const int32_t* unit_of;    // LINES: sampled-line index of (frame k, line l)
  int width, nx, r, kind, nchunks;
  int ngroups, ua;       // LINES: coil groups and lines allocated per group in P
  long npairs;           // LINES: pairs allocated per group in hp
  const double* ysq_k;
  float2* B;             // r x q
  float2* B_out;         // non-null: B also written here (the caller's buffer)
  float2* bcp;           // LINES: conj(b_k) per pair, for the gradient fold
  double* cost_k;
  DevState* st;
  int check_halt;
};

struct BasisArgs {
  const float2* U;       // n x r basis, pixel-major [p][j]
  float2* W;             // [c][row][x][j]
  float2* K;             // [c][row][x][j]
  float2* G;             // [part][p][j]
  const float2* coils;   // blocked [c][x / txx][y][x % txx]
  long n;
  int nx, r, nc, ua, txx, cgs;
  long part_stride;
  const int32_t* rows;        // sampled rows (ky) of W / K, or null: all rows
  const int32_t* n_rows_ptr;
  const int32_t* row_unit;    // k-space row -> row of W / K (-1: not kept), or null: identity
  const float2* tw;           // twiddles along y
  const float2* tw_x;         // twiddles along x
  float scale, scale_x;
  DevState* st;
  int check_halt;
  float2* qpart;              // k_adj_qr: the column's QR Gram partial (FP32, tri order)
};

struct PdftArgs {
  const float2* U;       // pixel-major [p][j]
  const float2* coils;   // [c][p]
  float2* W;             // [c][u][x][j], ua rows per coil (forward out)
  const float2* K;       // [c][u][x][j] (adjoint in)
  float2* G;             // [part][p][j] (adjoint out)
  const float2* tw;      // exp(-2 pi i t / ny), t < ny
  const int32_t* unit_loc;  // sampled row u -> ky
  int nx, r, nc, ua, cgs;
  long n, part_stride;
  float scale;           // 1 / sqrt(ny)
  DevState* st;
  int check_halt;
};

// warm-start CNN
struct ConvArgs {
  const float* X;        // [b][cin][H][W]
  const float* Wp;       // packed weights [kappa][32], kappa = tap*cin + ci, then the bias row
  float* Y;              // [b][cout][H][W]
  const float* mask;     // optional [b][cout][H][W]: Y = 0 where mask <= 0
  int cin, cout, H, W, bias, relu;
};

struct WgradArgs {
  const float* X;        // layer input [b][cin][H][W]
  const float* dY;       // gradient at the layer output [b][cout][H][W]
  float* part;           // [b][band][kp][32] partial weight gradients
  int cin, cout, H, W, kp, rows_per_band;
};

struct LossArgs {
  const float* Y4;       // network output [b][2r][n]
  const float2* Ut;      // targets [b][r][n] (column-major n x r)
  double2* part;         // [b][chunk][tri(2r)] Gram partials of [M Ut]
  double2* P;            // [b][2][r][r]: C^H G^-1, G^-1 C C^H G^-1
  double* loss_b;        // [b]
  float* dY4;            // [b][2r][n]
  long n, chunk;
  int r, nchunks;
  float scale;           // 1 / batch
};

struct FoldArgs {
  const int4* line_order;  // LINES: per fold row position (line u, first pair, pair count, 0), most pairs first; n_loc entries
  const float2* bcp;      // LINES: conj(b_k) of every pair, in pair order (written by the solve)
  const float2* W;
  const float2* yu;      // LINES: per-line data [c][p][x]
  const float2* y;       // INDEX: measurements
  const float2* B;
  const int2* pairs;
  const int32_t* loc_ptr;
  int nc, r, nx, ua, n, m_max;
  int max_pairs;         // at most this many frames sample one line or location (q)
  float2* K;
  DevState* st;
  int check_halt;
};

struct GramColsArgs {
  const float2* A;
  const float2* B;
  int m1, m2;
  long n;
  long rows_per_block;
  int nparts;            // B is the sum of nparts arrays at stride part_stride
  long part_stride;
  int write_sum;         // store the summed B back into part 0
  int a_colmajor;        // A is column-major n x m1 (else pixel-major [p][j])
  double2* part;         // per workgroup: its partial Gram (the QR Gram of FP32 MFMA stores float2 pairs)
  DevState* st;
  int check_halt;
};

struct QrSmallArgs {
  const double2* part;   // per QR Gram workgroup: its partial (FP32 pairs when part_f32)
  int part_f32;
  int nblk, r, mode, n, q;
  double eta_c, eta_cap_c, eps_exit;
  int exit_consec;  // the exit rule fires after this many consecutive small steps (>= 1)
  double guard;          // stationary start: ||grad_0||_2 <= guard * sum_k ||y_k||^2
  const float2* B;
  const double* cost_k;
  float2* rfac;          // R = L^H (Uhat^H Uhat = L L^H), row-major r x r, upper, 1 / R_jj on the diagonal
  DevState* st;
  int check_halt;
  int commit_direct;     // fused step only: workgroup 0 commits t and eta itself (the exit rule is off)
  double2* stats_src;    // fused step with commit_direct: the r x r inputs of the deferred statistics (193 entries)
};

struct ApplyArgs {
  float2* U;             // n x r column-major (C ABI layout)
  float2* Ui;            // n x r pixel-major copy for the next iteration (may be null)
  const float2* G;       // pixel-major gradient
  const float2* rfac;    // R as written by the small QR step
  float2* U_prev;
  long n;
  int r, mode;
  DevState* st;
};

struct InitEigArgs {
  const double2* part;
  int nblk, q, r;
  double2* V;            // 2 q x (q | 1) scratch (global): matrix and reflectors when not in LDS
  int in_lds;            // matrix and eigenvectors in dynamic LDS (q <= 64)
  float2* Vs;            // q x r out: V_r Sigma_r^{-1}
  double* lam_out;       // non-null: the r largest eigenvalues (descending) go here, no eigenvectors
  DevState* st;
};

__device__ __forceinline__ void set_error(DevState* st, int code, int frame) {
  if (atomicCAS(&st->err, 0, code) == 0) st->err_frame = frame;
  st->halt = 1;
}

// ---------------------------------------------------------------------------
// one-wave helpers for the small factorizations: a single wave works on
// registers and LDS with no workgroup barrier (lane = threadIdx.x & 63)
// ---------------------------------------------------------------------------
// value of v in lane src (src uniform)
__device__ __forceinline__ float lane_get(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_get(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float2 lane_get(float2 v, int src) { return make_float2(lane_get(v.x, src), lane_get(v.y, src)); }
__device__ __forceinline__ double2 lane_get(double2 v, int src) {
  return make_double2(lane_get(v.x, src), lane_get(v.y, src));
}
// v from another lane by a DPP move (CTRL: quad_perm / row_ror / row_half_mirror)
template <int CTRL>
__device__ __forceinline__ double dpp_get(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_getf(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
#define DPP_XOR1 0xB1       // quad_perm [1,0,3,2]
#define DPP_XOR2 0x4E       // quad_perm [2,3,0,1]
#define DPP_ROR4 0x124      // row_ror:4
#define DPP_ROR8 0x128      // row_ror:8
#define DPP_HALF_MIRROR 0x141
// maximum over the 64 lanes (every lane active)
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_get<DPP_XOR1>(v));
  v = fmax(v, dpp_get<DPP_XOR2>(v));
  v = fmax(v, dpp_get<DPP_ROR4>(v));
  v = fmax(v, dpp_get<DPP_ROR8>(v));
  return fmax(fmax(lane_get(v, 0), lane_get(v, 16)), fmax(lane_get(v, 32), lane_get(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) { return -wave_max(-v); }
// sum over the 64 lanes (every lane active): sums within rows of 16 by DPP,
// then the four row sums
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_get<DPP_XOR1>(v);
  v += dpp_get<DPP_XOR2>(v);
  v += dpp_get<DPP_ROR4>(v);
  v += dpp_get<DPP_ROR8>(v);
  return (lane_get(v, 0) + lane_get(v, 16)) + (lane_get(v, 32) + lane_get(v, 48));
}
// this wave's LDS writes are seen by its later LDS reads in any lane
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// complex helpers over float2 / double2
__device__ __forceinline__ float2 cx_mul(float2 a, float2 b) { return cmul(a, b); }
__device__ __forceinline__ double2 cx_mul(double2 a, double2 b) { return dmul(a, b); }
__device__ __forceinline__ float2 cx_cjm(float2 a, float2 b) { return cjmul(a, b); }    // conj(a) b
__device__ __forceinline__ double2 cx_cjm(double2 a, double2 b) { return djmul(a, b); }
__device__ __forceinline__ float2 cx_sub(float2 a, float2 b) { return csub(a, b); }
__device__ __forceinline__ double2 cx_sub(double2 a, double2 b) { return dsub(a, b); }
__device__ __forceinline__ float2 cx_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cx_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// reciprocal square root: the hardware estimate, refined by Newton steps in FP64
__device__ __forceinline__ float cx_rsqrt(float d) { return rsqrtf(d); }
__device__ __forceinline__ double cx_rsqrt(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

// Cholesky G = L L^H of a Hermitian positive definite RT x RT matrix by one
// wave: lane i < RT holds row i of G in g[0..RT-1] on entry and row i of L
// (entries 0..i) on return.  A problem of size r < RT is padded with the
// identity (rows and columns r..RT-1), so the code is straight-line and
// short.  False if a pivot of the r x r problem is not above tol (all lanes
// agree).
template <typename T, typename T2, int RT>
__device__ __forceinline__ bool wave_chol(T2 (&g)[RT], int r, T tol) {
  const int i = threadIdx.x & 63;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    const T d = lane_get(g[j].x, j);
    ok = ok && (j >= r || ((d > tol) && isfinite((double)d)));  // padding pivots are 1
    const T inv = cx_rsqrt(d > (T)0 ? d : (T)1), ljj = (d > (T)0 ? d : (T)1) * inv;
    if (i == j) {
      g[j].x = ljj;
      g[j].y = (T)0;
    } else if (i > j) {
      g[j] = cx_scale(g[j], inv);
    }
#pragma unroll
    for (int k = j + 1; k < RT; ++k) {
      const T2 lkj = lane_get(g[j], k);
      if (i >= k) g[k] = cx_sub(g[k], cx_mul(g[j], T2{lkj.x, -lkj.y}));
    }
  }
  return ok;
}

__device__ __forceinline__ void tri_index(int o, int r, int& i, int& j) {
  i = 0;
  int rem = o;
  while (rem >= r - i) {
    rem -= r - i;
    ++i;
  }
  j = i + rem;
}

__global__ void k_inv_bitmap(const int32_t* mask, const int32_t* m_k, int width, int per, int n_loc,
                             uint32_t* bitmap, int nw, DevState* st);
__global__ void k_inv_scan(const uint32_t* bitmap, int nw, int n_loc, int32_t* loc_ptr, int32_t* loc2unit,
                           int32_t* unit_loc, int2* unit_span, DevState* st);
__global__ void k_inv_fill(const int32_t* mask, const int32_t* m_k, int width, int per, const uint32_t* bitmap,
                           int nw, const int32_t* loc_ptr, const int32_t* loc2unit, int2* pairs, int32_t* pair_of,
                           int32_t* unit_of, const DevState* st);
__global__ void k_ysq(const float2* y, const int32_t* m_k, int nc, int m_max, double* part);
__global__ void k_ysq_sum(const double* part, int q, int nc, double* ysq_k);
__global__ void k_init_stats(const double* ysq_k, const int32_t* m_k, int q, double trunc_c, DevState* st);
__global__ void k_state_reset(DevState* st, int full);
__global__ void k_state_set_eta(DevState* st, double eta);
hipError_t launch_x_times_v(const float2* X, const float2* Vs, int n, int q, int r, float2* U, const DevState* st,
                            hipStream_t s);  // U = X0 Vs, r <= 16
__global__ void k_err_snapshot(const DevState* st, int32_t* snap);
__global__ void k_pick_init(const double* f, const int32_t* snap, const float2* src, float2* dst, long n,
                            int32_t* choice, const DevState* st);
__global__ void k_err_restore(const int32_t* snap, DevState* st);
__global__ void k_copy(const float2* src, float2* dst, long n);
__global__ void k_cost_total(const double* cost_k, int q, double* out, DevState* st);
__global__ void k_init_eig(InitEigArgs a);

hipError_t launch_gram_lines(const GramLinesArgs& a, int ny, int ngroups, int max_pairs, bool fp64,
                             hipStream_t s);
hipError_t launch_gram_index(const GramIndexArgs& a, int q, bool fp64, hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, int q, bool fp64, hipStream_t s);
hipError_t launch_gram_cols(const GramColsArgs& a, int nblk, bool fp64, hipStream_t s);
hipError_t launch_qr_gram(const GramColsArgs& a, int nblk, bool fp64, hipStream_t s);
hipError_t launch_init_gram(const GramColsArgs& a, int nblk, hipStream_t s);  // X0^H X0, q <= 48
hipError_t launch_init_gram_cx(const GramColsArgs& a, int nblk, hipStream_t s);  // X0^H X0, 48 < q <= 128
__global__ void k_sum_parts(const float2* src, long stride, int nparts, float2* dst, long n);
hipError_t launch_apply(const ApplyArgs& a, hipStream_t s);
hipError_t launch_basis(int which, int N, const BasisArgs& a, int grid_x, int grid_y, hipStream_t s);
hipError_t launch_adj_qr(int N, const BasisArgs& a, hipStream_t s);
hipError_t launch_fold2(const FoldArgs& a, bool lines, int grid_x, int grid_y, hipStream_t s);
hipError_t launch_gram_work(const int2* unit_span, int4* items, int4* line_order, int n_loc, DevState* st,
                            hipStream_t s);
__global__ void k_build_yg(const float2* yu, const int4* items, int nc, int nx, float2* yg, const DevState* st);
hipError_t launch_cnn_pack(const float* Wl, int cin, int cout, int kp, int kpb, float* Wf, float* Wb, hipStream_t s);
hipError_t launch_conv(const ConvArgs& a, int batch, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs& a, int bands, int batch, int nparam_layer, float* g, float scale,
                        hipStream_t s);
hipError_t launch_loss(const LossArgs& a, int batch, double* d_loss, hipStream_t s);
hipError_t launch_cnn_to_M(const float* Y4, int r, long n, int batch, float2* M, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, int step, hipStream_t s);
hipError_t launch_cnn_planes(const float2* X, long n, int q, double* partial, float* out, hipStream_t s);
// mixed form, 1D Cartesian masks: which 0 forward, 1 adjoint + coil combine
hipError_t launch_pdft(int which, int ny, const PdftArgs& a, int grid_x, int grid_y, hipStream_t s);
int basis_txx(int N, int nx, int r);
__global__ void k_coil_block(const float2* coils, float2* dst, int nx, int ny, int txx, long n, int nc);
__global__ void k_build_yu(const float2* yh, const int2* pairs, const int32_t* mask, const int32_t* loc_ptr,
                           int n_loc, int width, int nc, int nx, int lmax, float2* yu, const DevState* st);
__global__ void k_to_colmajor(const float2* src, int r, long n, float2* dst);
__global__ void k_to_pixmajor(const float2* src, int r, long n, float2* dst);
hipError_t launch_qr_small(const QrSmallArgs& a, hipStream_t s);
hipError_t launch_init_eig(const InitEigArgs& a, hipStream_t s);
hipError_t launch_partials_total(const double2* part, int f32, int nblk, int nout, double2* total, hipStream_t s);
hipError_t launch_step_apply(const QrSmallArgs& a, const ApplyArgs& ap, hipStream_t s);
hipError_t launch_stats_finish(DevState* st, const double2* src, const double* cost_k, int q, int r, hipStream_t s);
hipError_t launch_sum_partials(const double2* part, int nblk, int nout, double2* out, hipStream_t s);

}  // namespace ag
