// Internal: the context behind the C ABI of include/altgdmin.h, shared by
// the translation units of the host side (the altGDmin loop in altgdmin.hip,
// the steps around it in mri.hip).  Not part of the public interface.
#pragma once

#include <vector>

#include "../../include/altgdmin.h"
#include "kernels_core.hpp"

using namespace ag;

enum TimedKernel {
  TK_NONE = 0,
  TK_FWD = 1,
  TK_GRAM = 2,
  TK_SOLVE = 3,
  TK_FOLD = 4,
  TK_ADJ = 5,
  TK_QRGRAM = 6,
  TK_QRSMALL = 7,
  TK_APPLY = 8,
  TK_COUNT = 9
};

struct altgdmin_ctx {
  altgdmin_params p;
  int n, lines, fp64;
  int pdft;       // ky transforms as FP16 hi+lo MFMA partial DFTs (mixed form, 1D Cartesian)
  int width;     // mask row width: lines per frame (LINES) or m_max (INDEX)
  int lmax;      // LINES: m_max / nx
  int per;       // samples per mask entry (nx for LINES, 1 for INDEX)
  int n_loc, nw;
  int ua;        // rows per (c, j) plane of W / K
  int nchunks;   // INDEX gram chunks per frame
  int qr_nblk;
  long qr_rows;
  int kc;        // INDEX: frames per chunk of the operator passes
  int gram_cg, gram_ngroups, gram_chunk;
  int adj_parts, adj_cgs;  // coil groups of the basis transforms (the adjoint's partial gradients)
  int adj_qr;              // 1: the adjoint sums every coil and forms the QR Gram partials (k_adj_qr)
  // set by altgdmin_iterate for the duration of one call: the caller's B
  // buffer, which every solve writes too
  float2* b_out;
  int grad_parts;          // partial gradient arrays the adjoint writes
  int txx;                 // image columns per workgroup in the basis transforms
  size_t bytes;
  // bound problem
  const float2* coils = nullptr;
  const int32_t* mask = nullptr;
  const int32_t* m_k = nullptr;
  const float2* y = nullptr;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int bound = 0, initialized = 0;
  // workspace carve
  size_t o_st, o_twx, o_twy, o_bitmap, o_locptr, o_loc2unit, o_unitloc, o_pairs, o_pairof, o_yh, o_ysq,
      o_cost, o_W, o_K, o_P, o_hp, o_B, o_G, o_qpart, o_qtot, o_rfac, o_Vs, o_V, o_T, o_Ui, o_unitof, o_unitspan, o_bcp, o_Uc,
      o_fcmp, o_planes, o_gwork, o_lineord, o_coilb, o_yg, o_ysqp, o_stsrc, o_end;
  size_t T_bytes;
  // timing
  int timed = TK_NONE;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;

  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  DevState* st() const { return at<DevState>(o_st); }
};

#define HIPCHK(x)                               \
  do {                                          \
    hipError_t _e = (x);                        \
    if (_e != hipSuccess) return ALTGDMIN_EHIP; \
  } while (0)

// host-side pieces of altgdmin.hip that the other host translation units use
namespace ag_host {
// X = A^H(Y) (n x q, column-major), scaled per column by 1/sqrt(m_k mbar)
// when scale_mk, with the truncation of Algorithm 2 when trunc
hipError_t adjoint_op(altgdmin_ctx* c, const float2* Y, float2* X, int trunc, int scale_mk);
// Y = A(X) in the padded measurement layout
hipError_t forward_op(altgdmin_ctx* c, const float2* X, float2* Y);
// the truncated back-projection X_0 (into the workspace) and the top r_eig
// eigenpairs of X_0^H X_0: eigenvalues to lam_out (device, descending) when
// it is non-null (then no eigenvectors), else V_r Sigma_r^-1 for the context's r
hipError_t spectral_eig(altgdmin_ctx* c, int r_eig, double* lam_out);
inline altgdmin_status map_hip(hipError_t e) { return e == hipSuccess ? ALTGDMIN_OK : ALTGDMIN_EHIP; }
}  // namespace ag_host
