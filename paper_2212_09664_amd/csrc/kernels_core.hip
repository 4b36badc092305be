// altGDmin kernels other than the transforms: the inverse sampling map,
// per-frame Gram / right-hand side (the LS step of Algorithm 2), the batched
// r x r Cholesky solves, the gradient fold, the Gram of the QR step, the
// small dense r x r / q x q work (Cholesky, triangular inverse, Jacobi
// eigensolver) and the spectral-initialisation helpers.
#include "kernels_core.hpp"

namespace ag {


// ===========================================================================
// setup: inverse sampling map
// A "location" is a phase-encode line ky (LINES) or a flat k-space index
// (INDEX).  For every location the list of (frame k, position e) samples
// that hit it is stored contiguously, in increasing k (deterministic).
// ===========================================================================
__global__ void k_inv_bitmap(const int32_t* mask, const int32_t* m_k, int width, int per, int n_loc,
                             uint32_t* bitmap, int nw, DevState* st) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
  const int mk = m_k[k];
  if (mk < 0 || mk > width * per || (mk % per) != 0) {
    if (e == 0) set_error(st, 1 /*EINVAL: bad m_k*/, k);
    return;
  }
  if (e >= mk / per) return;
  const int loc = mask[(long)k * width + e];
  if (loc < 0 || loc >= n_loc) {
    set_error(st, 1 /*EINVAL*/, k);
    return;
  }
  const uint32_t bit = 1u << (k & 31);
  const uint32_t old = atomicOr(&bitmap[(long)loc * nw + (k >> 5)], bit);
  if (old & bit) set_error(st, 1 /*EINVAL: repeated location in a frame*/, k);
}

// the locations' sample counts and their exclusive prefix sums (pairs per
// location), and the sampled locations (units) numbered in order; one block
// of 1024 threads over tiles of 1024 locations, scans within waves by
// shuffles, a running total across tiles
__global__ __launch_bounds__(1024) void k_inv_scan(const uint32_t* bitmap, int nw, int n_loc,
                                                   int32_t* loc_ptr, int32_t* loc2unit,
                                                   int32_t* unit_loc, int2* unit_span, DevState* st) {
  constexpr int LPT = 1;  // locations per thread and tile (4: slower, the loads less coalesced)
  __shared__ int s_wc[16], s_wu[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry_c = 0, carry_u = 0;  // totals of the tiles before this one
  for (int base = 0; base < n_loc; base += 1024 * LPT) {
    const int l0 = base + LPT * tid;
    int cs[LPT], tc = 0, tu = 0;
#pragma unroll
    for (int s2 = 0; s2 < LPT; ++s2) {
      const int l = l0 + s2, lc = min(l, n_loc - 1);
      int c = 0;
      for (int w = 0; w < nw; ++w) c += __popc(bitmap[(long)lc * nw + w]);
      cs[s2] = l < n_loc ? c : 0;
      tc += cs[s2];
      tu += cs[s2] > 0;
    }
    int sc = tc, su = tu;  // inclusive scans over the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int vc = __shfl_up(sc, off), vu = __shfl_up(su, off);
      if (lane >= off) {
        sc += vc;
        su += vu;
      }
    }
    if (lane == 63) {
      s_wc[wv] = sc;
      s_wu[wv] = su;
    }
    __syncthreads();
    int pc = carry_c + sc - tc, pu = carry_u + su - tu;  // exclusive prefixes of this thread's first location
    for (int w2 = 0; w2 < 16; ++w2) {
      const int vc = s_wc[w2], vu = s_wu[w2];
      if (w2 < wv) {
        pc += vc;
        pu += vu;
      }
      carry_c += vc;
      carry_u += vu;
    }
#pragma unroll
    for (int s2 = 0; s2 < LPT; ++s2) {
      const int l = l0 + s2, c = cs[s2];
      if (l < n_loc) {
        loc_ptr[l] = pc;
        if (c > 0) {
          loc2unit[l] = pu;
          unit_loc[pu] = l;
          unit_span[pu] = make_int2(pc, c);  // the unit's samples: pairs [pc, pc + c)
          ++pu;
        } else {
          loc2unit[l] = -1;
        }
      }
      pc += c;
    }
    __syncthreads();  // the wave totals are read before the next tile writes them
  }
  if (tid == 0) {
    loc_ptr[n_loc] = carry_c;
    st->n_units = carry_u;
  }
}

__global__ void k_inv_fill(const int32_t* mask, const int32_t* m_k, int width, int per,
                           const uint32_t* bitmap, int nw, const int32_t* loc_ptr, const int32_t* loc2unit,
                           int2* pairs, int32_t* pair_of, int32_t* unit_of, const DevState* st) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
  if (st->err) return;
  if (e >= m_k[k] / per) return;
  const int loc = mask[(long)k * width + e];
  const uint32_t* bm = bitmap + (long)loc * nw;
  int rank = 0;
  for (int w = 0; w < (k >> 5); ++w) rank += __popc(bm[w]);
  rank += __popc(bm[k >> 5] & ((1u << (k & 31)) - 1u));
  const int pos = loc_ptr[loc] + rank;
  pairs[pos] = make_int2(k, e);
  pair_of[(long)k * width + e] = pos;
  unit_of[(long)k * width + e] = loc2unit[loc];
}

// ||y_{k,c}||^2 in FP64, one workgroup per (frame k, coil c): part[k * nc + c]
__global__ __launch_bounds__(AG_NT) void k_ysq(const float2* y, const int32_t* m_k, int nc, int m_max,
                                               double* part) {
  __shared__ double red[AG_NT];
  const int k = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const int mk = m_k[k];
  const float2* yk = y + ((long)k * nc + c) * m_max;
  double s = 0.0;
#pragma unroll 8
  for (int i = tid; i < mk; i += AG_NT) {
    const float2 v = yk[i];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[tid] = s;
  __syncthreads();
  for (int off = AG_NT / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) part[(long)k * nc + c] = red[0];
}

// ||y_k||^2 = sum over coils of the parts, in coil order (one thread per frame)
__global__ void k_ysq_sum(const double* part, int q, int nc, double* ysq_k) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < q; k += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += part[(long)k * nc + c];
    ysq_k[k] = s;
  }
}

// gamma = trunc_c * sum |y|^2 / (m q), m = max_k m_k; mbar = sum_k m_k / q
__global__ void k_init_stats(const double* ysq_k, const int32_t* m_k, int q, double trunc_c, DevState* st) {
  if (threadIdx.x != 0) return;
  double ys = 0.0, msum = 0.0;
  int mmax = 0;
  for (int k = 0; k < q; ++k) {
    ys += ysq_k[k];
    msum += m_k[k];
    mmax = max(mmax, m_k[k]);
  }
  st->ysq = ys;
  st->mbar = msum / q;
  st->gamma = trunc_c > 0 ? trunc_c * ys / ((double)mmax * q) : INFINITY;
}

__global__ void k_state_reset(DevState* st, int full) {
  if (threadIdx.x != 0) return;
  if (full) {
    st->err = 0;
    st->err_frame = -1;
    st->n_units = 0;
    st->n_gwork = 0;
  }
  st->halt = 0;
  st->step_ok = 0;
  st->t = 0;
  st->exited = 0;
  st->converged = 0;
  st->eta = -1.0;
  st->step_flags = 0;
  st->eta_next = -1.0;
  st->f = 0.0;
  st->sd = 0.0;
  st->grad_norm = 0.0;
  st->stats_pending = 0;
  st->n_trunc = 0;
  st->exit_run = 0;
}

__global__ void k_state_set_eta(DevState* st, double eta) {
  if (threadIdx.x == 0) st->eta = eta;
}

// ===========================================================================
// per-frame Gram and right-hand side, 1D Cartesian (hybrid ky, x form)
// For each sampled line (unit u, phase-encode ky):
//   P_u  = sum_{c,x} W_c(u,x,:)^H W_c(u,x,:)                  (r x r)
//   hp_p = sum_{c,x} conj(W_c(u,x,:)) y'_{k,c}(l,x)            per sample (k,l) of ky
// so that G_k = sum_{l} P_{u(k,l)} and h_k = sum_l hp_{(k,l)}.
// Rows of W_c(u,:,:) and the samples' y' rows are staged in LDS; every
// thread owns a few outputs and forms their dot products over x.
// ===========================================================================

template <typename ACC>
struct Acc2;
template <>
struct Acc2<float> {
  using T = float2;
  __device__ static T zero() { return make_float2(0.f, 0.f); }
  __device__ static T fma_cj(T acc, float2 a, float2 b) {  // acc + conj(a) b
    acc.x += a.x * b.x + a.y * b.y;
    acc.y += a.x * b.y - a.y * b.x;
    return acc;
  }
  __device__ static double2 to_d(T v) { return f2d(v); }
};
template <>
struct Acc2<double> {
  using T = double2;
  __device__ static T zero() { return make_double2(0.0, 0.0); }
  __device__ static T fma_cj(T acc, float2 a, float2 b) {
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    acc.x += ax * bx + ay * by;
    acc.y += ax * by - ay * bx;
    return acc;
  }
  __device__ static double2 to_d(T v) { return v; }
};

// ===========================================================================
// Gram of column blocks: C = [A B]^H [A B] over n rows (column-major n x m1
// and n x m2), upper triangle, partial sums per workgroup in FP64.
// ===========================================================================
template <typename ACC>
__global__ __launch_bounds__(GCOLS_NT) void k_gram_cols(GramColsArgs a) {
  using A2 = Acc2<ACC>;
  __shared__ float2 Xs[64 * 64];
  const int tid = threadIdx.x, blk = blockIdx.x;
  if (halted(a.st, a.check_halt)) return;
  const int m = a.m1 + a.m2;  // <= 128
  const int nout = m * (m + 1) / 2;
  const int RC = m <= 64 ? 64 : 32;  // rows staged per chunk
  typename A2::T acc[GCOLS_OPT];
#pragma unroll
  for (int t = 0; t < GCOLS_OPT; ++t) acc[t] = A2::zero();
  const long pa = (long)blk * a.rows_per_block;
  const long pb = min((long)a.n, pa + a.rows_per_block);
  for (long p0 = pa; p0 < pb; p0 += RC) {
    const int np = (int)min((long)RC, pb - p0);
    for (int g = tid; g < RC * m; g += GCOLS_NT) {
      const int j = g / RC, pp = g % RC;
      float2 v = make_float2(0.f, 0.f);
      if (pp < np) v = (j < a.m1) ? a.A[(long)j * a.n + p0 + pp] : a.B[(long)(j - a.m1) * a.n + p0 + pp];
      Xs[pp * m + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < GCOLS_OPT; ++t) {
      const int o = tid + t * GCOLS_NT;
      if (o < nout) {
        int i, j;
        tri_index(o, m, i, j);
        for (int pp = 0; pp < np; ++pp) acc[t] = A2::fma_cj(acc[t], Xs[pp * m + i], Xs[pp * m + j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < GCOLS_OPT; ++t) {
    const int o = tid + t * GCOLS_NT;
    if (o < nout) a.part[(long)blk * nout + o] = A2::to_d(acc[t]);
  }
}

// ===========================================================================
// small dense FP64 routines for one workgroup (matrices in LDS, leading
// dimension ld).
// ===========================================================================
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  double s = red[0];
  __syncthreads();
  return s;
}

// one complex Jacobi rotation G (c, s, e) that zeroes A[p][q] of the
// Hermitian 2x2 block [[app, apq], [conj(apq), aqq]]; identity if q >= n or
// the entry is already negligible
// reciprocal and reciprocal square root in FP64 from the hardware estimates
// (v_rcp_f64, v_rsq_f64) refined by two Newton steps each, to about one ulp:
// shorter dependent chains than the IEEE-exact division and square root
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

__device__ __forceinline__ JRot jacobi_rot(const double2* A, int ld, int n, int p, int q) {
  JRot g{1.0, 0.0, make_double2(1.0, 0.0)};
  if (q >= n) return g;
  const double2 apq = A[p * ld + q];
  const double m2 = apq.x * apq.x + apq.y * apq.y;
  const double app = A[p * ld + p].x, aqq = A[q * ld + q].x;
  const double scale = fabs(app) + fabs(aqq);
  if (m2 > 1e-280 && m2 > 1e-36 * scale * scale) {
    const double rm = rsq_nr(m2);  // 1 / |a_pq|
    g.e = make_double2(apq.x * rm, -apq.y * rm);  // exp(-i phi)
    const double tau = (aqq - app) * 0.5 * rm;
    const double at = fabs(tau);
    // t = sign(tau) / (|tau| + sqrt(1 + tau^2)); for huge |tau|, t ~ 1 / (2 tau)
    const double h = (at < 1e150) ? (1.0 + tau * tau) * rsq_nr(1.0 + tau * tau) : at;
    const double t = (tau >= 0 ? 1.0 : -1.0) * rcp_nr(at + h);
    g.c = rsq_nr(1.0 + t * t);
    g.s = t * g.c;
  }
  return g;
}

// pair i of round s of the round-robin ordering over Q (even) indices
__device__ __forceinline__ void jacobi_pair(int s, int i, int Q, int& p, int& q) {
  if (i == 0) {
    p = Q - 1;
    q = s;
  } else {
    p = (s + i) % (Q - 1);
    q = (s - i + Q - 1) % (Q - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Cyclic complex Jacobi eigensolver for the Hermitian n x n matrix A
// (row-major, leading dimension ld), parallel round-robin ordering: the
// Q/2 rotations of a round are disjoint and are applied together.  The
// matrix splits into 2x2 blocks (pair i rows, pair j columns); each block
// is updated independently, A_ij <- G_i^H A_ij G_j, with the rotations
// computed first (one thread per pair) from the matrix as it was at the
// start of the round; then a read phase and a write phase.  V (if given, ld n) accumulates
// V <- V G in place (block (i, j) of V is touched by one thread only).  A and V may be in LDS or in global memory private to the
// workgroup.  On return diag(A) holds the eigenvalues and the columns of V
// the eigenvectors.  Up to ITEMS*blockDim blocks: ITEMS = 1 covers n <= 64
// with 1024 threads, ITEMS = 4 covers n <= 128.
//
// With r_top > 0 only the invariant subspace of the r_top largest
// eigenvalues is wanted.  Partition the indices into the current top r_top
// diagonal entries and the rest, A = [A11 A12; A21 A22].  Gershgorin discs
// within each diagonal block bound the spectra of A11 from below and of A22
// from above; once these bounds are separated by sep > 0 and
// ||A12||_F <= 1e-10 sep, the span of the top coordinate vectors is within
// an angle of about 1e-10 of the wanted subspace (Davis-Kahan sin-theta),
// and the sweeps stop.
template <int JAC_ITEMS>
__device__ __forceinline__ void jacobi_eig(double2* A, int n, int ld, double2* V, JacobiScratch* js,
                                           int max_sweeps, int r_top = 0) {
  const int tid = threadIdx.x, NT = blockDim.x;
  if (V)
    for (int e = tid; e < n * n; e += NT) V[e] = make_double2((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  const int Q = n + (n & 1), H = Q / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (r_top > 0) {  // which diagonal entries are currently the top r_top
      for (int i = tid; i < n; i += NT) {
        const double di = A[i * ld + i].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
          const double dj = A[j * ld + j].x;
          rank += (dj > di) || (dj == di && j < i);
        }
        js->top[i] = rank < r_top;
      }
      __syncthreads();
      // Gershgorin bound of row i within its own block
      for (int i = tid; i < n; i += NT) {
        const int ti = js->top[i];
        double rad = 0.0;
        for (int j = 0; j < n; ++j) {
          if (j == i || js->top[j] != ti) continue;
          const double2 v = A[i * ld + j];
          rad += fabs(v.x) + fabs(v.y);  // >= |v|: still a Gershgorin bound
        }
        js->bnd[i] = ti ? A[i * ld + i].x - rad : A[i * ld + i].x + rad;
      }
      __syncthreads();
    }
    double off = 0.0, tot = 0.0, cross = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const int i = e / n, j = e % n;
      const double2 v = A[i * ld + j];
      const double m2 = v.x * v.x + v.y * v.y;
      tot += m2;
      if (i != j) off += m2;
      if (r_top > 0 && js->top[i] && !js->top[j]) cross += m2;
    }
    off = block_sum(off, js->red);
    tot = block_sum(tot, js->red);
    if (!(off > 1e-26 * tot)) break;
    if (r_top > 0 && r_top < n) {
      cross = block_sum(cross, js->red);
      double lo = INFINITY, hi = -INFINITY;  // lower bound of eig(A11), upper bound of eig(A22)
      for (int i = 0; i < n; ++i) {
        if (js->top[i]) lo = fmin(lo, js->bnd[i]);
        else hi = fmax(hi, js->bnd[i]);
      }
      const double sep = lo - hi;
      if (sep > 0.0 && cross <= 1e-20 * sep * sep) break;
    }
    for (int s = 0; s < Q - 1; ++s) {
      // this round's rotations, one thread per pair, from the matrix as it is
      for (int i = tid; i < H; i += NT) {
        int p, q;
        jacobi_pair(s, i, Q, p, q);
        js->rot[i] = jacobi_rot(A, ld, n, p, q);
        js->pq[i] = make_int2(p, q);
      }
      __syncthreads();
      double2 na[JAC_ITEMS][4];
#pragma unroll
      for (int k = 0; k < JAC_ITEMS; ++k) {
        const int t = tid + k * NT;
        if (t < H * H) {
          const int i = t / H, j = t - (t / H) * H;
          const int pi = js->pq[i].x, qi = js->pq[i].y, pj = js->pq[j].x, qj = js->pq[j].y;
          const JRot gi = js->rot[i];
          const JRot gj = js->rot[j];
          const bool ri = qi < n, rj = qj < n;  // the second row / column exists
          const double2 z = make_double2(0.0, 0.0);
          // the block [[a, b], [c, d]] = A[(pi, qi), (pj, qj)]
          double2 a = A[pi * ld + pj], b = rj ? A[pi * ld + qj] : z;
          double2 c = ri ? A[qi * ld + pj] : z, d = (ri && rj) ? A[qi * ld + qj] : z;
          // columns: (x, y) <- (c x - s y e, s x + c y e)
          {
            const double2 y0 = dmul(b, gj.e), y1 = dmul(d, gj.e);
            const double2 a2 = make_double2(gj.c * a.x - gj.s * y0.x, gj.c * a.y - gj.s * y0.y);
            const double2 b2 = make_double2(gj.s * a.x + gj.c * y0.x, gj.s * a.y + gj.c * y0.y);
            const double2 c2 = make_double2(gj.c * c.x - gj.s * y1.x, gj.c * c.y - gj.s * y1.y);
            const double2 d2 = make_double2(gj.s * c.x + gj.c * y1.x, gj.s * c.y + gj.c * y1.y);
            a = a2; b = b2; c = c2; d = d2;
          }
          // rows: with conj(e_i)
          {
            const double2 ec = dconj(gi.e);
            const double2 y0 = dmul(c, ec), y1 = dmul(d, ec);
            na[k][0] = make_double2(gi.c * a.x - gi.s * y0.x, gi.c * a.y - gi.s * y0.y);
            na[k][1] = make_double2(gi.c * b.x - gi.s * y1.x, gi.c * b.y - gi.s * y1.y);
            na[k][2] = make_double2(gi.s * a.x + gi.c * y0.x, gi.s * a.y + gi.c * y0.y);
            na[k][3] = make_double2(gi.s * b.x + gi.c * y1.x, gi.s * b.y + gi.c * y1.y);
          }
          if (V) {  // V rows (pi, qi), columns (pj, qj), right rotation only: no other
                    // thread touches these entries this round, so update in place
            const double2 va = V[pi * n + pj], vb = rj ? V[pi * n + qj] : z;
            const double2 vc = ri ? V[qi * n + pj] : z, vd = (ri && rj) ? V[qi * n + qj] : z;
            const double2 y0 = dmul(vb, gj.e), y1 = dmul(vd, gj.e);
            V[pi * n + pj] = make_double2(gj.c * va.x - gj.s * y0.x, gj.c * va.y - gj.s * y0.y);
            if (rj) V[pi * n + qj] = make_double2(gj.s * va.x + gj.c * y0.x, gj.s * va.y + gj.c * y0.y);
            if (ri) V[qi * n + pj] = make_double2(gj.c * vc.x - gj.s * y1.x, gj.c * vc.y - gj.s * y1.y);
            if (ri && rj) V[qi * n + qj] = make_double2(gj.s * vc.x + gj.c * y1.x, gj.s * vc.y + gj.c * y1.y);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < JAC_ITEMS; ++k) {
        const int t = tid + k * NT;
        if (t < H * H) {
          const int i = t / H, j = t - (t / H) * H;
          const int pi = js->pq[i].x, qi = js->pq[i].y, pj = js->pq[j].x, qj = js->pq[j].y;
          const bool ri = qi < n, rj = qj < n;
          A[pi * ld + pj] = na[k][0];
          if (rj) A[pi * ld + qj] = na[k][1];
          if (ri) A[qi * ld + pj] = na[k][2];
          if (ri && rj) A[qi * ld + qj] = na[k][3];
        }
      }
      __syncthreads();
    }
  }
}

// Cholesky of the Hermitian r x r matrix M (LDS, ld 16) in FP64, lower L in
// place, right-looking, by the whole workgroup (every thread must call it).
// Returns false (in every thread) if M is not positive definite.
__device__ bool chol_lower(double2* M, int r) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double dmax = 0.0;
  for (int i = 0; i < r; ++i) dmax = fmax(dmax, M[i * 16 + i].x);
  for (int j = 0; j < r; ++j) {
    const double d = M[j * 16 + j].x;  // every thread reads the same pivot
    if (!(d > 1e-14 * dmax) || !isfinite(d)) return false;
    const double ljj = sqrt(d), inv = 1.0 / ljj;
    __syncthreads();
    if (tid == 0) M[j * 16 + j] = make_double2(ljj, 0.0);
    for (int i = j + 1 + tid; i < r; i += nt) M[i * 16 + j] = make_double2(M[i * 16 + j].x * inv, M[i * 16 + j].y * inv);
    __syncthreads();
    // trailing update of the lower triangle: M[i][k] -= L[i][j] conj(L[k][j]), j < k <= i
    for (int e = tid; e < 256; e += nt) {
      const int i = e >> 4, k = e & 15;
      if (k > j && k <= i && i < r) M[i * 16 + k] = dsub(M[i * 16 + k], dmul(M[i * 16 + j], dconj(M[k * 16 + j])));
    }
    __syncthreads();
  }
  return true;
}

// entry e = (i, j) of R = L^H with the reciprocal on the diagonal, from the
// lower Cholesky factor L (LDS, ld 16): the form the update kernel solves with
__device__ __forceinline__ float2 rfac_entry(const double2* L, int r, int e) {
  const int i = e / r, j = e - (e / r) * r;
  if (i < j) return make_float2((float)L[j * 16 + i].x, -(float)L[j * 16 + i].y);
  if (i == j) return make_float2((float)(1.0 / L[i * 16 + i].x), 0.f);
  return make_float2(0.f, 0.f);
}

// ===========================================================================
// the QR step's small work (one workgroup): reduce the Gram partials of
// [U grad]; at the first iteration set eta = eta_c / sigma_max(grad) (with
// the stationarity guard and the optional cap); Gram of Uhat = U - eta grad
// from the blocks; R = chol(.)^H, R^{-1}; SD(U, U+) from r x r data.
// mode 1: plain CholeskyQR of U (no gradient).
// ===========================================================================
template <int RT>
__global__ __launch_bounds__(1024) void k_qr_small(QrSmallArgs a) {
  __shared__ double2 UU[256], UG[256], GG[256], Gh[256], Tm[256];
  __shared__ JacobiScratch js;
  __shared__ int s_ok;
  const int tid = threadIdx.x, r = a.r;
  DevState* st = a.st;
  if (st->err || (a.mode == 0 && a.check_halt && st->halt)) {
    if (tid == 0 && a.mode == 0) st->step_ok = 0;
    return;
  }
  const int m = a.mode == 1 ? r : 2 * r;  // mode 0 step, 1 CholeskyQR of U, 2 step size only
  const int nout = m * (m + 1) / 2;
  // sum the block partials: thread = (output, slice of blocks)
  __shared__ double2 red2[1024];
  const int NTH = blockDim.x;
  const int NS = max(1, NTH / nout);
  const int OW = NTH / NS;
  for (int o0 = 0; o0 < nout; o0 += OW) {
    const int o = o0 + tid % OW, sl = tid / OW;
    double2 s = make_double2(0.0, 0.0);
    if (o < nout && sl < NS) {
      if (a.part_f32) {
        const float2* pf = reinterpret_cast<const float2*>(a.part);
#pragma unroll 8
        for (int b = sl; b < a.nblk; b += NS) s = dadd(s, f2d(pf[(long)b * nout + o]));
      } else {
#pragma unroll 8
        for (int b = sl; b < a.nblk; b += NS) s = dadd(s, a.part[(long)b * nout + o]);
      }
    }
    red2[tid] = s;
    __syncthreads();
    if (tid < OW && o < nout) {
      for (int q2 = 1; q2 < NS; ++q2) s = dadd(s, red2[tid + q2 * OW]);
      int i, j;
    tri_index(o, m, i, j);
    // entry (i, j), i <= j, of [U G]^H [U G]
    if (j < r) {
      UU[i * 16 + j] = s;
      UU[j * 16 + i] = dconj(s);
    } else if (i < r) {
      UG[i * 16 + (j - r)] = s;  // (U^H G)[i][j-r]
    } else {
      GG[(i - r) * 16 + (j - r)] = s;
      GG[(j - r) * 16 + (i - r)] = dconj(s);
    }
    }
    __syncthreads();
  }
  __syncthreads();
  if (a.mode == 1) {
    for (int e = tid; e < 256; e += blockDim.x) Gh[e] = UU[e];
    __syncthreads();
    bool ok = chol_lower(Gh, r);
    __syncthreads();
    if (!ok) {  // numerically rank-deficient basis: retry with a small ridge
      for (int e = tid; e < 256; e += blockDim.x) Gh[e] = UU[e];
      __syncthreads();
      double tr = 0.0;
      for (int i = 0; i < r; ++i) tr += UU[i * 16 + i].x;
      __syncthreads();
      if (tid < r) Gh[tid * 16 + tid].x += 1e-6 * tr / r;
      __syncthreads();
      ok = (tr > 0.0) && isfinite(tr) && chol_lower(Gh, r);
      __syncthreads();
    }
    if (!ok) {
      if (tid == 0) set_error(st, 4, -1);
      return;
    }
    for (int e = tid; e < r * r; e += blockDim.x) a.rfac[e] = rfac_entry(Gh, r, e);
    return;
  }
  // first iteration: step size from the spectral norm of grad
  if (st->eta <= 0.0) {
    for (int e = tid; e < 256; e += AG_NT) Tm[e] = GG[e];
    __syncthreads();
    jacobi_eig<1>(Tm, r, 16, nullptr, &js, 40);
    __syncthreads();
    if (tid == 0) {
      double lam = 0.0;
      for (int i = 0; i < r; ++i) lam = fmax(lam, Tm[i * 16 + i].x);
      const double smax = sqrt(lam);
      st->grad_norm = smax;
      if (!(smax > a.guard * st->ysq)) {
        st->converged = 1;
        st->halt = 1;
        st->step_ok = 0;
        s_ok = 0;
      } else {
        st->eta = a.eta_c / smax;
        s_ok = 1;
      }
    }
    __syncthreads();
    if (!s_ok) return;
    if (a.eta_cap_c > 0.0) {  // cap: eta <= c n / (mbar ||B_0||_2^2)
      for (int e = tid; e < r * r; e += AG_NT) {
        const int i = e / r, j = e % r;
        double2 s = make_double2(0.0, 0.0);
        for (int k = 0; k < a.q; ++k) s = dadd(s, dmul(f2d(a.B[(long)k * r + i]), dconj(f2d(a.B[(long)k * r + j]))));
        Tm[i * 16 + j] = s;
      }
      __syncthreads();
      jacobi_eig<1>(Tm, r, 16, nullptr, &js, 40);
      __syncthreads();
      if (tid == 0) {
        double lam = 0.0;
        for (int i = 0; i < r; ++i) lam = fmax(lam, Tm[i * 16 + i].x);
        const double cap = a.eta_cap_c * (double)a.n / (st->mbar * lam);
        if (cap < st->eta) st->eta = cap;
      }
      __syncthreads();
    }
  }
  if (a.mode == 2) return;  // only the step size was wanted
  // the step size as thread 0 left it, shared through LDS
  __shared__ double s_eta;
  if (tid == 0) s_eta = st->eta;
  __syncthreads();
  // one wave from here on: Cholesky of Uhat^H Uhat, Uhat = U - eta G, from the
  // blocks (rows in lanes), R^{-1}, SD(U, U+) and the cost
  if (tid >= 64) return;
  const int i = tid;
  const double eta = s_eta;
  auto gh = [&](int a_, int b_) -> double2 {  // (Uhat^H Uhat)[a_][b_]
    const double2 ug = UG[a_ * 16 + b_], gu = dconj(UG[b_ * 16 + a_]);
    const double2 v = UU[a_ * 16 + b_], g = GG[a_ * 16 + b_];
    return make_double2(v.x - eta * (ug.x + gu.x) + eta * eta * g.x, v.y - eta * (ug.y + gu.y) + eta * eta * g.y);
  };
  double2 g[RT];  // padded to RT with the identity
#pragma unroll
  for (int m = 0; m < RT; ++m) g[m] = (i < r && m < r) ? gh(i, m) : make_double2(i == m ? 1.0 : 0.0, 0.0);
  const double dmax = wave_max((i < r) ? gh(i, i).x : 0.0);
  if (!wave_chol<double, double2, RT>(g, r, 1e-14 * dmax)) {
    if (i == 0) {
      set_error(st, 4, -1);
      st->step_ok = 0;
    }
    return;
  }
#pragma unroll
  for (int m = 0; m < RT; ++m)
    if (i < RT && m <= i) Gh[i * 16 + m] = g[m];
  wave_sync();
  // U^H U+ = (U^H U - eta U^H G) R^{-1}: lane i solves x R = row i by forward
  // substitution (R = L^H); SD^2 = r - ||U^H U+||_F^2
  double fro = 0.0;
  if (i < r) {  // x in LDS (Tm, free after the first iteration's step size): short code, few registers
    double2* x = Tm + i * 16;
    for (int j = 0; j < r; ++j) {
      double2 acc = make_double2(UU[i * 16 + j].x - eta * UG[i * 16 + j].x, UU[i * 16 + j].y - eta * UG[i * 16 + j].y);
      for (int k = 0; k < j; ++k) acc = dsub(acc, dmul(x[k], dconj(Gh[j * 16 + k])));  // R[k][j] = conj(L[j][k])
      const double rd = 1.0 / Gh[j * 16 + j].x;
      const double2 xj = make_double2(acc.x * rd, acc.y * rd);
      x[j] = xj;
      fro += xj.x * xj.x + xj.y * xj.y;
    }
  }
  fro = wave_sum(fro);
  for (int e = i; e < r * r; e += 64) a.rfac[e] = rfac_entry(Gh, r, e);
  double fv = 0.0;  // f = sum_k cost_k
  for (int k = i; k < a.q; k += 64) fv += a.cost_k[k];
  fv = wave_sum(fv);
  if (i == 0) {
    const double sd2 = fmax(0.0, (double)r - fro);
    double tr = 0.0;
    for (int m = 0; m < r; ++m) tr += GG[m * 16 + m].x;
    st->sd = sqrt(sd2);
    st->grad_norm = sqrt(tr);
    st->f = fv;
    st->t += 1;
    st->step_ok = 1;
    if (a.eps_exit > 0.0 && sqrt(sd2 / r) < a.eps_exit) {
      st->exit_run += 1;
      if (st->exit_run >= a.exit_consec) {
        st->exited = 1;
        st->halt = 1;
      }
    } else {
      st->exit_run = 0;
    }
  }
}

// U <- (U - eta grad) Rinv per pixel (mode 0, when the step is applied), or
// U <- U Rinv (mode 1).  Optionally keeps U before the update.
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_apply(ApplyArgs a) {
  __shared__ float2 Ri[RT * RT];
  const int tid = threadIdx.x;
  const long p = (long)blockIdx.x * AG_NT + tid;
  const int r = a.r;
  // this pixel's basis row and gradient are requested before the state is
  // read (clamped addresses, valid either way)
  const long pc = min(p, a.n - 1);
  float2 u0[RT], g0[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    u0[i] = (i < r) ? a.U[(long)i * a.n + pc] : make_float2(0.f, 0.f);
    g0[i] = (i < r && a.mode == 0) ? a.G[pc * r + i] : make_float2(0.f, 0.f);  // gradient is pixel-major
  }
  for (int e = tid; e < r * r; e += AG_NT) Ri[(e / r) * RT + (e % r)] = a.rfac[e];
  if (a.mode == 0 && !a.st->step_ok) return;
  if (a.st->err) return;
  __syncthreads();
  if (p >= a.n) return;
  const float eta = (a.mode == 0) ? (float)a.st->eta : 0.f;
  float2 uh[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    if (i < r) {
      if (a.U_prev) a.U_prev[(long)i * a.n + p] = u0[i];
      uh[i] = make_float2(u0[i].x - eta * g0[i].x, u0[i].y - eta * g0[i].y);
    } else {
      uh[i] = make_float2(0.f, 0.f);
    }
  }
  // U+ R = Uhat, row by row: forward substitution (the diagonal holds 1 / R_jj)
  float2 un[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    un[j] = make_float2(0.f, 0.f);
    if (j < r) {
      float2 s = uh[j];
#pragma unroll
      for (int i = 0; i < j; ++i) s = csub(s, cmul(un[i], Ri[i * RT + j]));
      un[j] = cscale(s, Ri[j * RT + j].x);
      a.U[(long)j * a.n + p] = un[j];
      if (a.Ui) a.Ui[p * r + j] = un[j];
    }
  }
}

// ===========================================================================
// spectral initialisation: eigen-decomposition of X_0^H X_0 (q x q) and the
// scaled top-r eigenvectors V_r Sigma_r^{-1}, so that X_0 V_r Sigma_r^{-1}
// are the top-r left singular vectors of X_0.
// ===========================================================================
// IN_LDS: matrix and eigenvectors in dynamic LDS (q <= 64; the accesses are
// then LDS instructions), else in the workspace
// ||U^H U+||_F^2 = ||(U^H U - eta U^H G) R^{-1}||_F^2, lanes l < r taking
// row l by forward substitution with R = L^H (L in Gh, rows of stride 16;
// x is a row scratch of stride 16); the caller sums over the wave.  The
// fused step and the deferred statistics both use it, so that SD is the
// same number either way.
__device__ __forceinline__ double sd_row_sum(const double2* UU, const double2* UG, const double2* Gh, double2* Tm,
                                             double eta, int r, int l) {
  double fro = 0.0;
  if (l < r) {
    double2* x = Tm + l * 16;
    for (int j = 0; j < r; ++j) {
      double2 acc = make_double2(UU[l * 16 + j].x - eta * UG[l * 16 + j].x, UU[l * 16 + j].y - eta * UG[l * 16 + j].y);
      for (int k = 0; k < j; ++k) acc = dsub(acc, dmul(x[k], dconj(Gh[j * 16 + k])));
      const double rd = 1.0 / Gh[j * 16 + j].x;
      const double2 xj = make_double2(acc.x * rd, acc.y * rd);
      x[j] = xj;
      fro += xj.x * xj.x + xj.y * xj.y;
    }
  }
  return fro;
}

// ---------------------------------------------------------------------------
// tot[o] = sum over the nblk QR Gram partials (FP32 pairs when f32, else
// FP64) of nout complex entries, in FP64; workgroup wg of nwg takes a range
// of the 16-byte units (one or two entries).  Thread = (unit, slice): slice
// sl sums partials sl, sl + NS, sl + 2 NS, ... in that order, with PL loads
// in flight (issued from clamped, valid addresses before any is used), and
// the slices are then added in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void unit_add(double2& a0, double2&, const double2 w) { a0 = dadd(a0, w); }
__device__ __forceinline__ void unit_add(double2& a0, double2&, const float2 w) { a0 = dadd(a0, f2d(w)); }
__device__ __forceinline__ void unit_add(double2& a0, double2& a1, const float4 w) {
  a0 = dadd(a0, make_double2(w.x, w.y));
  a1 = dadd(a1, make_double2(w.z, w.w));
}

template <int PL, typename L>
__device__ __forceinline__ void slice_sum(const L* src, int nblk, int nunit, int u, int sl, int NS, double2& a0,
                                          double2& a1) {
  for (int b0 = sl; b0 < nblk; b0 += NS * PL) {
    L w[PL];
#pragma unroll
    for (int k = 0; k < PL; ++k) w[k] = src[(long)min(b0 + k * NS, nblk - 1) * nunit + u];
#pragma unroll
    for (int k = 0; k < PL; ++k)
      if (b0 + k * NS < nblk) unit_add(a0, a1, w[k]);
  }
}

template <int NT>
__device__ __forceinline__ void partials_sum(const double2* part, int f32, int nblk, int nout, double2* tot, int wg,
                                             int nwg) {
  constexpr int PL = 16;
  static_assert(NT <= 256, "16 loads of 16 bytes in flight per thread need more than 1024-thread workgroups allow");
  __shared__ double2 s_sum[2][NT];
  const int tid = threadIdx.x;
  const int per = (f32 && (nout & 1) == 0) ? 2 : 1;  // outputs per load
  const int nunit = nout / per, cu = (nunit + nwg - 1) / nwg, ub = wg * cu, ue = min(nunit, ub + cu);
  const int nu = max(0, ue - ub);
  const int NS = max(1, min(32, NT / max(nu, 1))), OW = NT / NS;  // (at most 32 slices: their sum is serial)
  for (int u0 = 0; u0 < nu; u0 += OW) {
    const int u = ub + u0 + tid % OW, sl = tid / OW, uc = min(u, ue - 1);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0;
    if (sl < NS) {
      if (!f32) slice_sum<PL>(part, nblk, nunit, uc, sl, NS, a0, a1);
      else if (per == 2) slice_sum<PL>(reinterpret_cast<const float4*>(part), nblk, nunit, uc, sl, NS, a0, a1);
      else slice_sum<PL>(reinterpret_cast<const float2*>(part), nblk, nunit, uc, sl, NS, a0, a1);
    }
    s_sum[0][tid] = a0;
    s_sum[1][tid] = a1;
    __syncthreads();
    if (sl == 0 && u < ue) {
      for (int q = 1; q < NS; ++q) {
        a0 = dadd(a0, s_sum[0][tid + q * OW]);
        a1 = dadd(a1, s_sum[1][tid + q * OW]);
      }
      tot[u * per] = a0;
      if (per == 2) tot[u * per + 1] = a1;
    }
    __syncthreads();
  }
}

// ===========================================================================
// the QR step fused with the update (r <= 8): every workgroup sums the QR
// Gram partials, takes the step size (Algorithm 2's rule at t = 1, then the
// stored one), factors Uhat^H Uhat = L L^H in one wave, and solves
// U+ R = U - eta grad for its NT pixels, R = L^H.  Every workgroup computes
// the same factor from the same partials in the same order.  With the exit
// rule on, workgroup 0 also forms SD(U, U+) and the cost, and the outcome
// (applied, exit rule, stationary start) and the step size go to step_flags /
// eta_next and are committed by k_step_commit, because a halt written during
// the launch would stop workgroups that have not yet updated their pixels.
// With it off (commit_direct), workgroup 0 commits t and eta itself: t is
// read by no workgroup, and a workgroup that reads the new eta instead of the
// unset one gets the value it would have computed (the same rule on the same
// partials, bitwise); the stationary start halts every workgroup alike.  SD,
// the cost and ||grad|| are then only reported: their r x r inputs are
// stored and k_stats_finish forms them on request.
// ===========================================================================
template <int RT, int NT>
__global__ __launch_bounds__(NT) void k_step_apply(QrSmallArgs a, ApplyArgs ap) {
  __shared__ double2 UU[256], UG[256], GG[256], Gh[256], Tm[256];
  __shared__ JacobiScratch js;
  __shared__ double2 tot[RT * (2 * RT + 1)];  // the summed Gram's upper triangle (m = 2 r <= 2 RT)
  __shared__ float2 Rf[RT * RT];
  __shared__ int s_ok;
  __shared__ double s_eta;
  const int tid = threadIdx.x, r = a.r, wv = tid >> 6, l = tid & 63;
  DevState* st = a.st;
  const long n = ap.n, p = (long)blockIdx.x * NT + tid, pc = min(p, n - 1);
  // the state, then this pixel's basis row and gradient, requested first
  // (clamped, valid addresses); the state's loads are in every thread, so
  // that no branch waits on them
  const int err0 = st->err;
  const int halt0 = __hip_atomic_load(&st->halt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double eta0 = __hip_atomic_load(&st->eta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 u0[RT], g0[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) u0[i] = (i < r) ? ap.U[(long)i * n + pc] : make_float2(0.f, 0.f);
  if (r == RT) {  // the pixel-major gradient row as 16-byte loads
    const float4* gs = reinterpret_cast<const float4*>(ap.G + pc * RT);
#pragma unroll
    for (int h = 0; h < RT / 2; ++h) {
      const float4 w = gs[h];
      g0[2 * h] = make_float2(w.x, w.y);
      g0[2 * h + 1] = make_float2(w.z, w.w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < RT; ++i) g0[i] = (i < r) ? ap.G[pc * r + i] : make_float2(0.f, 0.f);
  }
  // the Gram of [U G] from the partials
  const int m = 2 * r, nout = m * (m + 1) / 2;
  const bool summed = a.nblk == 1 && !a.part_f32;  // the FP64 sum itself
  if (!summed) partials_sum<NT>(a.part, a.part_f32, a.nblk, nout, tot, 0, 1);
  for (int o = tid; o < nout; o += NT) {
    int i, j;
    tri_index(o, m, i, j);
    const double2 sum = summed ? a.part[o] : tot[o];
    if (j < r) {
      UU[i * 16 + j] = sum;
      UU[j * 16 + i] = dconj(sum);
    } else if (i < r) {
      UG[i * 16 + (j - r)] = sum;
    } else {
      GG[(i - r) * 16 + (j - r)] = sum;
      GG[(j - r) * 16 + (i - r)] = dconj(sum);
    }
  }
  __syncthreads();
  // err is written during this launch only when a factor fails, which then
  // fails in every workgroup alike; halt and eta only by workgroup 0, with
  // the values every workgroup derives itself (see above)
  if (tid == 0) {
    s_ok = !(err0 || (a.check_halt && halt0));
    s_eta = eta0;
  }
  __syncthreads();
  if (!s_ok) return;
  if (!(s_eta > 0.0)) {  // first iteration: eta = eta_c / ||grad||_2 (with the guard and the cap)
    for (int e = tid; e < 256; e += NT) Tm[e] = GG[e];
    __syncthreads();
    jacobi_eig<1>(Tm, r, 16, nullptr, &js, 40);
    __syncthreads();
    if (tid == 0) {
      double lam = 0.0;
      for (int i = 0; i < r; ++i) lam = fmax(lam, Tm[i * 16 + i].x);
      const double smax = sqrt(lam);
      if (!(smax > a.guard * st->ysq)) {
        s_ok = 0;  // stationary start
        if (blockIdx.x == 0) {
          st->grad_norm = smax;
          if (a.commit_direct) {
            st->converged = 1;
            __hip_atomic_store(&st->halt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            st->step_flags = STEP_CONVERGED;
          }
        }
      } else {
        s_eta = a.eta_c / smax;
      }
    }
    __syncthreads();
    if (!s_ok) return;
    if (a.eta_cap_c > 0.0) {  // cap: eta <= c n / (mbar ||B_0||_2^2)
      for (int e = tid; e < r * r; e += NT) {
        const int i = e / r, j = e % r;
        double2 sum = make_double2(0.0, 0.0);
        for (int k = 0; k < a.q; ++k)
          sum = dadd(sum, dmul(f2d(a.B[(long)k * r + i]), dconj(f2d(a.B[(long)k * r + j]))));
        Tm[i * 16 + j] = sum;
      }
      __syncthreads();
      jacobi_eig<1>(Tm, r, 16, nullptr, &js, 40);
      __syncthreads();
      if (tid == 0) {
        double lam = 0.0;
        for (int i = 0; i < r; ++i) lam = fmax(lam, Tm[i * 16 + i].x);
        const double cap = a.eta_cap_c * (double)a.n / (st->mbar * lam);
        if (cap < s_eta) s_eta = cap;
      }
      __syncthreads();
    }
  }
  const double eta = s_eta;
  if (wv == 0) {  // one wave: the Cholesky factor (rows in lanes, padded with the identity)
    auto gh = [&](int a_, int b_) -> double2 {  // (Uhat^H Uhat)[a_][b_]
      const double2 ug = UG[a_ * 16 + b_], gu = dconj(UG[b_ * 16 + a_]);
      const double2 v = UU[a_ * 16 + b_], g = GG[a_ * 16 + b_];
      return make_double2(v.x - eta * (ug.x + gu.x) + eta * eta * g.x, v.y - eta * (ug.y + gu.y) + eta * eta * g.y);
    };
    double2 g[RT];
#pragma unroll
    for (int mm = 0; mm < RT; ++mm) g[mm] = (l < r && mm < r) ? gh(l, mm) : make_double2(l == mm ? 1.0 : 0.0, 0.0);
    const double dmax = wave_max((l < r) ? gh(l, l).x : 0.0);
    const bool ok = wave_chol<double, double2, RT>(g, r, 1e-14 * dmax);
    if (!ok) {
      if (l == 0) {
        s_ok = 0;
        set_error(st, 4, -1);
      }
    } else {
#pragma unroll
      for (int mm = 0; mm < RT; ++mm)
        if (l < RT && mm <= l) Gh[l * 16 + mm] = g[mm];
      wave_sync();
      for (int e = l; e < r * r; e += 64) Rf[(e / r) * RT + (e % r)] = rfac_entry(Gh, r, e);
      if (blockIdx.x == 0) {
        if (a.commit_direct) {
          // exit rule off: SD, f and ||grad|| are only reported; their r x r
          // inputs are stored and k_stats_finish forms them when asked
          for (int e = l; e < 64; e += 64) {
            const int i = e >> 3, j = e & 7;
            a.stats_src[e] = UU[i * 16 + j];
            a.stats_src[64 + e] = UG[i * 16 + j];
            a.stats_src[128 + e] = Gh[i * 16 + j];
          }
          if (l == 0) {
            double tr = 0.0;
            for (int mm = 0; mm < r; ++mm) tr += GG[mm * 16 + mm].x;
            a.stats_src[192] = make_double2(eta, tr);
            st->stats_pending = 1;
            __hip_atomic_store(&st->eta, eta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st->t += 1;
            st->step_ok = 1;
          }
        } else {
          // SD^2 = r - ||U^H U+||_F^2 decides the exit rule
          const double fro = wave_sum(sd_row_sum(UU, UG, Gh, Tm, eta, r, l));
          double fv = 0.0;  // f = sum_k cost_k
          for (int k = l; k < a.q; k += 64) fv += a.cost_k[k];
          fv = wave_sum(fv);
          if (l == 0) {
            const double sd2 = fmax(0.0, (double)r - fro);
            double tr = 0.0;
            for (int mm = 0; mm < r; ++mm) tr += GG[mm * 16 + mm].x;
            st->sd = sqrt(sd2);
            st->grad_norm = sqrt(tr);
            st->f = fv;
            st->stats_pending = 0;
            st->eta_next = eta;
            st->step_flags = STEP_APPLIED | ((a.eps_exit > 0.0 && sqrt(sd2 / r) < a.eps_exit) ? STEP_EXIT : 0);
          }
        }
      }
    }
  }
  __syncthreads();
  if (!s_ok || p >= n) return;
  // U+ R = U - eta grad for this pixel (forward substitution, 1 / R_jj on the diagonal)
  const float etaf = (float)eta;
  float2 un[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    un[j] = make_float2(0.f, 0.f);
    if (j < r) {
      if (ap.U_prev) ap.U_prev[(long)j * n + p] = u0[j];
      float2 sv = make_float2(u0[j].x - etaf * g0[j].x, u0[j].y - etaf * g0[j].y);
#pragma unroll
      for (int i = 0; i < j; ++i) sv = csub(sv, cmul(un[i], Rf[i * RT + j]));
      un[j] = cscale(sv, Rf[j * RT + j].x);
      ap.U[(long)j * n + p] = un[j];
      if (ap.Ui && r != RT) ap.Ui[p * r + j] = un[j];
    }
  }
  if (ap.Ui && r == RT) {  // the pixel-major row as 16-byte stores
    float4* dst = reinterpret_cast<float4*>(ap.Ui + p * RT);
#pragma unroll
    for (int h = 0; h < RT / 2; ++h) dst[h] = make_float4(un[2 * h].x, un[2 * h].y, un[2 * h + 1].x, un[2 * h + 1].y);
  }
}

// the fused step's outcome into the state (one thread, after it)
__global__ void k_step_commit(DevState* st, int exit_consec) {
  if (threadIdx.x != 0) return;
  const int f = st->step_flags;
  st->step_flags = 0;
  st->step_ok = 0;
  if (st->err) return;
  if (f & STEP_CONVERGED) {
    st->converged = 1;
    st->halt = 1;
  } else if (f & STEP_APPLIED) {
    st->eta = st->eta_next;
    st->t += 1;
    st->step_ok = 1;
    if (f & STEP_EXIT) {
      st->exit_run += 1;
      if (st->exit_run >= exit_consec) {
        st->exited = 1;
        st->halt = 1;
      }
    } else {
      st->exit_run = 0;
    }
  }
}

// the statistics the fused step left pending (exit rule off): SD, f and
// ||grad||_F of the last applied step, from its r x r inputs and the
// per-frame costs (no solve has run since), with the fused step's own code
__global__ __launch_bounds__(64) void k_stats_finish(DevState* st, const double2* src, const double* cost_k, int q,
                                                     int r) {
  __shared__ double2 UU[256], UG[256], Gh[256], Tm[256];
  const int l = threadIdx.x;
  if (!st->stats_pending) return;
  for (int e = l; e < 64; e += 64) {
    const int i = e >> 3, j = e & 7;
    UU[i * 16 + j] = src[e];
    UG[i * 16 + j] = src[64 + e];
    Gh[i * 16 + j] = src[128 + e];
  }
  const double2 et = src[192];
  wave_sync();
  const double fro = wave_sum(sd_row_sum(UU, UG, Gh, Tm, et.x, r, l));
  double fv = 0.0;
  for (int k = l; k < q; k += 64) fv += cost_k[k];
  fv = wave_sum(fv);
  if (l == 0) {
    st->sd = sqrt(fmax(0.0, (double)r - fro));
    st->grad_norm = sqrt(et.y);
    st->f = fv;
    st->stats_pending = 0;
  }
}

hipError_t launch_stats_finish(DevState* st, const double2* src, const double* cost_k, int q, int r, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_finish, dim3(1), dim3(64), 0, s, st, src, cost_k, q, r);
  return hipGetLastError();
}

// the QR Gram partials summed once for the fused step: workgroups of 256
// threads, each over a few 16-byte units, so that one round of loads covers
// its partials
__global__ __launch_bounds__(256) void k_partials_total(const double2* part, int f32, int nblk, int nout,
                                                        double2* total) {
  partials_sum<256>(part, f32, nblk, nout, total, blockIdx.x, gridDim.x);
}

hipError_t launch_partials_total(const double2* part, int f32, int nblk, int nout, double2* total, hipStream_t s) {
  const int per = (f32 && (nout & 1) == 0) ? 2 : 1, nunit = nout / per;
  // 8 units per workgroup: 32 slices of 16 loads in flight cover 512 partials
  const int nwg = (nunit + 7) / 8;
  hipLaunchKernelGGL(k_partials_total, dim3(nwg), dim3(256), 0, s, part, f32, nblk, nout, total);
  return hipGetLastError();
}

hipError_t launch_step_apply(const QrSmallArgs& a, const ApplyArgs& ap, hipStream_t s) {
  if (a.r > 8) return hipErrorInvalidValue;
  // 256 pixels per workgroup: the update's stores spread over every compute unit
  hipLaunchKernelGGL((k_step_apply<8, 256>), dim3((unsigned)((ap.n + 255) / 256)), dim3(256), 0, s, a, ap);
  if (!a.commit_direct) hipLaunchKernelGGL(k_step_commit, dim3(1), dim3(64), 0, s, a.st, a.exit_consec);
  return hipGetLastError();
}

// one-wave reductions
__device__ __forceinline__ double2 wave_sum2(double2 v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }

// number of eigenvalues of the real symmetric tridiagonal (d, e) below x
// (Sturm count of the LDL^T pivots; tiny pivots are replaced by -pivmin)
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
#pragma unroll 8
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// back-transformation by one wave (q <= 64): Y = Q D Z with Q = H_0 ... H_{n-3},
// then V_r Sigma_r^{-1} = Y diag(1 / sqrt(lambda_j)) into Vs (r <= RJ).  Lane
// (column j = l / G, row group g = l % G, G = 64 / RJ) keeps rows g, g + G, ... of Y in
// registers for the whole product; a reflector's column sums are taken over
// a column's G adjacent lanes by DPP moves, with no barrier; rows outside the
// reflector are selected to zero rather than branched around.
template <int RJ, int NR>
__device__ __forceinline__ void backtransform_wave(const double2* Vh, int ld, const double* s_beta, const double2* s_ph,
                                                   const double* sy, const double* s_lam, int n, int r, int l,
                                                   float2* Vs) {
  constexpr int G = 64 / RJ;
  static_assert(G == 4 || G == 8, "column sums over 4 or 8 adjacent lanes");
  const int j = l / G, g = l % G, jc = min(j, r - 1);
  double2 y[NR];
  int roff[NR];
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int i = g + G * t, ic = min(i, n - 1);
    roff[t] = ic * ld;
    const double z = i < n ? sy[ic * r + jc] : 0.0;
    const double2 ph = s_ph[ic];
    y[t] = make_double2(ph.x * z, ph.y * z);
  }
  for (int k = n - 3; k >= 0; --k) {
    const double beta = s_beta[k];
    if (beta == 0.0) continue;  // the same in every lane
    // the reflector's rows kept in registers when they fit (NR <= 8), else read again for the update
    constexpr bool KEEP = NR <= 8;
    double2 v[KEEP ? NR : 1];
    double sx = 0.0, sy_ = 0.0;
#pragma unroll
    for (int t = 0; t < NR; ++t) {  // conj(v) y over the reflector's rows
      // rows outside it read a valid address whose content is not the
      // reflector's (possibly not a finite number): selected away, not
      // multiplied by zero
      const int i = g + G * t;
      const double2 vl = Vh[roff[t] + k];
      const double2 vt = (i > k && i < n) ? vl : make_double2(0.0, 0.0);
      if constexpr (KEEP) v[t] = vt;
      sx = fma(vt.x, y[t].x, fma(vt.y, y[t].y, sx));
      sy_ = fma(vt.x, y[t].y, fma(-vt.y, y[t].x, sy_));
    }
    sx += dpp_get<DPP_XOR1>(sx);
    sy_ += dpp_get<DPP_XOR1>(sy_);
    sx += dpp_get<DPP_XOR2>(sx);
    sy_ += dpp_get<DPP_XOR2>(sy_);
    if constexpr (G == 8) {
      sx += dpp_get<DPP_HALF_MIRROR>(sx);
      sy_ += dpp_get<DPP_HALF_MIRROR>(sy_);
    }
    sx *= beta;
    sy_ *= beta;
#pragma unroll
    for (int t = 0; t < NR; ++t) {  // y -= v (beta v^H y), zero outside the reflector
      double2 vt;
      if constexpr (KEEP) {
        vt = v[t];
      } else {
        const int i = g + G * t;
        const double2 vl = Vh[roff[t] + k];
        vt = (i > k && i < n) ? vl : make_double2(0.0, 0.0);
      }
      const double ux = vt.x * sx - vt.y * sy_, uy = vt.x * sy_ + vt.y * sx;
      y[t] = make_double2(y[t].x - ux, y[t].y - uy);
    }
  }
  const double sc = 1.0 / sqrt(s_lam[jc]);
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int i = g + G * t;
    if (i < n && j < r) Vs[i * r + j] = make_float2((float)(y[t].x * sc), (float)(y[t].y * sc));
  }
}

// ===========================================================================
// spectral initialisation, the q x q eigenproblem: the r largest eigenpairs
// of the Hermitian X_0^H X_0 by one wave, then V_r Sigma_r^{-1}:
//  1. Householder reduction M = Q T Q^H, T tridiagonal with complex
//     off-diagonals e_k; reflectors H_k = I - beta_k v_k v_k^H kept in Vh;
//  2. a diagonal unitary D makes T real: T = D T_r D^H, off-diagonals |e_k|;
//  3. the r largest eigenvalues of T_r by multisection on Sturm counts;
//  4. their eigenvectors by inverse iteration (one lane each, LDL^T without
//     pivoting, tiny pivots replaced), orthogonalised within clusters;
//  5. back-transformation Y = Q D Z.
// IN_LDS: matrix and reflectors in dynamic LDS (q <= 64), else in the workspace.
// ===========================================================================
template <bool IN_LDS>
__global__ __launch_bounds__(1024) void k_init_eig(InitEigArgs a) {
  // q <= 64: the q x q matrix, then the q x q reflectors; 64 < q <= 128: the
  // matrix's lower triangle packed by rows (row i from i (i + 1) / 2), the
  // reflectors in global memory (a.V)
  extern __shared__ double2 lds_m[];
  __shared__ double s_d[128], s_ea[128], s_e2[128], s_beta[128];
  __shared__ double2 s_ec[128], s_ph[128], s_w[128], s_v[128];
  __shared__ double2 s_p[8][128];  // the reflector product's column-slice partials
  __shared__ double s_lam[16];
  __shared__ double s_gs[4];  // Gershgorin interval (lo, hi), the scale, the pivot floor
  const int tid = threadIdx.x, NT = blockDim.x, n = a.q, r = a.r;
  // row pitch ld odd: the rows one wave reads together fall in distinct LDS banks
  const int ld = n | 1;
  double2* A = lds_m;
  double2* Vh = IN_LDS ? A + n * ld : a.V;
  auto tri = [](int i) { return (i * (i + 1)) >> 1; };  // packed row offset
  const int nout = n * (n + 1) / 2;
  for (int o = tid; o < nout; o += NT) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll 16
    for (int b = 0; b < a.nblk; ++b) sum = dadd(sum, a.part[(long)b * nout + o]);
    int i, j;
    tri_index(o, n, i, j);
    if (i == j) sum.y = 0.0;
    if constexpr (IN_LDS) {
      A[i * ld + j] = sum;
      A[j * ld + i] = dconj(sum);
    } else {
      A[tri(max(i, j)) + min(i, j)] = i >= j ? sum : dconj(sum);  // the lower entry
    }
  }
  __syncthreads();
  // ---- 1. Householder tridiagonalisation (full Hermitian trailing block
  // kept): wave 0 forms each reflector, the workgroup shares the product
  // p = beta B v (8 column slices) and the rank-2 update of B
  const int l = tid & 63, wv = tid >> 6;
  if constexpr (IN_LDS) {
    for (int k = 0; k + 2 < n; ++k) {
      const int k1 = k + 1, m = n - k1;
      if (wv == 0) {
        double sig = 0.0;
        for (int i = 1 + l; i < m; i += 64) {
          const double2 x = A[(k1 + i) * ld + k];
          sig += x.x * x.x + x.y * x.y;
        }
        sig = wave_sum(sig);
        const double2 x0 = A[k1 * ld + k];
        if (sig == 0.0 && x0.y == 0.0) {  // already reduced: H_k = I
          if (l == 0) {
            s_beta[k] = 0.0;
            s_ec[k] = x0;
          }
        } else {
          const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y), nrm = sqrt(ax0 * ax0 + sig);
          const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
          const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
          const double2 v0 = dsub(x0, alpha);
          for (int i = 1 + l; i < m; i += 64) Vh[(k1 + i) * ld + k] = A[(k1 + i) * ld + k];
          if (l == 0) {
            Vh[k1 * ld + k] = v0;
            s_beta[k] = 2.0 / (v0.x * v0.x + v0.y * v0.y + sig);
            s_ec[k] = alpha;
          }
        }
      }
      __syncthreads();
      const double beta = s_beta[k];
      if (beta == 0.0) continue;  // the same in every thread
      // partial products over column slices j = h (mod 8), 8 waves
      if (wv < 8) {
  #pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          if (i < m) {
            const double2* row = A + (k1 + i) * ld + k1;
            double2 acc = make_double2(0.0, 0.0);
            for (int j = wv; j < m; j += 8) acc = dadd(acc, dmul(row[j], Vh[(k1 + j) * ld + k]));
            s_p[wv][i] = acc;
          }
        }
      }
      __syncthreads();
      // p = beta B v, K = (beta / 2) v^H p, w = p - K v (wave 0)
      if (wv == 0) {
        double2 pv[2];
        double2 kp = make_double2(0.0, 0.0);
  #pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          double2 acc = make_double2(0.0, 0.0);
          if (i < m) {
  #pragma unroll
            for (int h = 0; h < 8; ++h) acc = dadd(acc, s_p[h][i]);
            acc = make_double2(beta * acc.x, beta * acc.y);
            kp = dadd(kp, djmul(Vh[(k1 + i) * ld + k], acc));
          }
          pv[hh] = acc;
        }
        kp = wave_sum2(kp);
        const double2 K = make_double2(0.5 * beta * kp.x, 0.5 * beta * kp.y);
  #pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          if (i < m) s_w[i] = dsub(pv[hh], dmul(K, Vh[(k1 + i) * ld + k]));
        }
      }
      __syncthreads();
      // B -= v w^H + w v^H, entry by entry over the workgroup
      for (int e = tid; e < m * m; e += NT) {
        const int i = e / m, j = e - (e / m) * m;
        const double2 vi = Vh[(k1 + i) * ld + k], wi = s_w[i];
        const double2 vj = Vh[(k1 + j) * ld + k], wj = s_w[j];
        double2* aij = A + (k1 + i) * ld + k1 + j;
        *aij = dsub(*aij, dadd(dmul(vi, dconj(wj)), dmul(wi, dconj(vj))));
      }
      __syncthreads();
    }
  } else {
    // the same steps on the packed lower triangle: B(i, j) of the trailing
    // block is the stored entry for i >= j and the conjugate of (j, i) above;
    // the step's reflector is read from LDS (s_v), its global copy kept for
    // the back-transformation; the rank-2 update touches the lower triangle
    // only (rows i = w, w + 16, ... by wave, columns by lane)
    for (int k = 0; k + 2 < n; ++k) {
      const int k1 = k + 1, m = n - k1;
      if (wv == 0) {
        double sig = 0.0;
        for (int i = 1 + l; i < m; i += 64) {
          const double2 x = A[tri(k1 + i) + k];
          sig += x.x * x.x + x.y * x.y;
        }
        sig = wave_sum(sig);
        const double2 x0 = A[tri(k1) + k];
        if (sig == 0.0 && x0.y == 0.0) {  // already reduced: H_k = I
          if (l == 0) {
            s_beta[k] = 0.0;
            s_ec[k] = x0;
          }
        } else {
          const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y), nrm = sqrt(ax0 * ax0 + sig);
          const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
          const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
          const double2 v0 = dsub(x0, alpha);
          for (int i = 1 + l; i < m; i += 64) {
            const double2 x = A[tri(k1 + i) + k];
            s_v[i] = x;
            Vh[(k1 + i) * ld + k] = x;
          }
          if (l == 0) {
            s_v[0] = v0;
            Vh[k1 * ld + k] = v0;
            s_beta[k] = 2.0 / (v0.x * v0.x + v0.y * v0.y + sig);
            s_ec[k] = alpha;
          }
        }
      }
      __syncthreads();
      const double beta = s_beta[k];
      if (beta == 0.0) continue;  // the same in every thread
      if (wv < 8) {  // partial products over column slices j = wv (mod 8)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          if (i < m) {
            // one load per entry from a selected (valid) index, no branch:
            // row k1 + i's offset is fixed for the lane, row k1 + j's is
            // wave-uniform
            const int ti = tri(k1 + i) + k1;
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
            for (int j = wv; j < m; j += 8) {
              const int up = i < j;
              const double2 raw = A[up ? tri(k1 + j) + k1 + i : ti + j];
              const double2 bij = make_double2(raw.x, up ? -raw.y : raw.y);
              acc = dadd(acc, dmul(bij, s_v[j]));
            }
            s_p[wv][i] = acc;
          }
        }
      }
      __syncthreads();
      if (wv == 0) {  // p = beta B v, K = (beta / 2) v^H p, w = p - K v
        double2 pv[2];
        double2 kp = make_double2(0.0, 0.0);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          double2 acc = make_double2(0.0, 0.0);
          if (i < m) {
#pragma unroll
            for (int h = 0; h < 8; ++h) acc = dadd(acc, s_p[h][i]);
            acc = make_double2(beta * acc.x, beta * acc.y);
            kp = dadd(kp, djmul(s_v[i], acc));
          }
          pv[hh] = acc;
        }
        kp = wave_sum2(kp);
        const double2 K = make_double2(0.5 * beta * kp.x, 0.5 * beta * kp.y);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = l + 64 * hh;
          if (i < m) s_w[i] = dsub(pv[hh], dmul(K, s_v[i]));
        }
      }
      __syncthreads();
      for (int i = wv; i < m; i += NT / 64) {  // B -= v w^H + w v^H, lower triangle
        const double2 vi = s_v[i], wi = s_w[i];
        double2* row = A + tri(k1 + i) + k1;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int j = l + 64 * hh;
          if (j <= i) row[j] = dsub(row[j], dadd(dmul(vi, dconj(s_w[j])), dmul(wi, dconj(s_v[j]))));
        }
      }
      __syncthreads();
    }
  }
  if (wv == 0) {  // one wave: the tridiagonal eigenproblem
    // ---- 2. T_r: diagonal, |e_k|, and the phases of D
    for (int i = l; i < n; i += 64) s_d[i] = (IN_LDS ? A[i * ld + i] : A[tri(i) + i]).x;
    if (l == 0 && n >= 2) s_ec[n - 2] = IN_LDS ? A[(n - 1) * ld + (n - 2)] : A[tri(n - 1) + n - 2];
    wave_sync();
    for (int i = l; i + 1 < n; i += 64) {
      const double2 e = s_ec[i];
      const double ae = sqrt(e.x * e.x + e.y * e.y);
      s_ea[i] = ae;
      s_e2[i] = ae * ae;
    }
    if (l == 0) {
      double2 ph = make_double2(1.0, 0.0);
      s_ph[0] = ph;
      for (int i = 0; i + 1 < n; ++i) {
        const double2 e = s_ec[i];
        const double ae = sqrt(e.x * e.x + e.y * e.y);
        if (ae > 0.0) ph = dmul(ph, make_double2(e.x / ae, e.y / ae));
        s_ph[i + 1] = ph;
      }
    }
    wave_sync();
    // Gershgorin interval and scales
    double glo = INFINITY, ghi = -INFINITY, emax2 = 0.0, scale = 0.0;
    for (int i = l; i < n; i += 64) {
      const double rad = (i > 0 ? s_ea[i - 1] : 0.0) + (i + 1 < n ? s_ea[i] : 0.0);
      glo = fmin(glo, s_d[i] - rad);
      ghi = fmax(ghi, s_d[i] + rad);
      scale = fmax(scale, fabs(s_d[i]) + rad);
      if (i + 1 < n) emax2 = fmax(emax2, s_e2[i]);
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    scale = fmax(wave_max(scale), 1e-300);
    emax2 = wave_max(emax2);
    if (l == 0) {
      const double wdt = ghi - glo;
      s_gs[0] = glo - (1e-3 * wdt + 1e-300);
      s_gs[1] = ghi + (1e-3 * wdt + 1e-300);
      s_gs[2] = scale;
      s_gs[3] = 2.3e-308 * fmax(1.0, emax2);  // pivmin
    }
  }
  __syncthreads();
  // ---- 3. multisection: wave w < r takes the w-th largest eigenvalue
  // (ascending index n-1-w), its 64 lanes one Sturm count each per round (a
  // 65-section of the interval), to an isolating interval of relative width
  // 1e-10: inverse iteration converges from it and the Rayleigh quotient
  // refines the value
  const double scale = s_gs[2];
  if (wv < r) {
    const int idx = n - 1 - wv;
    const double pivmin = s_gs[3];
    double lo = s_gs[0], hi = s_gs[1];
    for (int rnd = 0; rnd < 80; ++rnd) {
      const double x = lo + (hi - lo) * (double)(l + 1) / 65.0;
      const int cnt = sturm_count(s_d, s_e2, n, x, pivmin);
      const double nlo = wave_max(cnt <= idx ? x : -INFINITY);
      const double nhi = wave_min(cnt > idx ? x : INFINITY);
      lo = fmax(lo, nlo);
      hi = fmin(hi, nhi);
      if (hi - lo <= 1e-10 * fmax(fabs(lo), fabs(hi)) + 1e-300) break;  // the same in every lane
    }
    if (l == 0) s_lam[wv] = 0.5 * (lo + hi);
  }
  __syncthreads();
  if (wv == 0) {
    // ---- 4. inverse iteration, lane j < r for eigenvalue j; scratch in A's region
    double* su = reinterpret_cast<double*>(A);  // u pivots [i * r + j]
    double* sy = su + n * r;                    // right-hand side / solution [i * r + j]
    if (l < r) {
      const double lam = s_lam[l], tiny = 1e-14 * scale;
      for (int i = 0; i < n; ++i) {  // a start vector of its own per lane (golden-ratio sequence)
        const double t = (double)(i + 1) * (double)(2 * l + 3) * 0.6180339887498949;
        sy[i * r + l] = 0.5 + (t - floor(t));
      }
      for (int it = 0; it < 3; ++it) {
        double u = s_d[0] - lam, y = sy[l];
  #pragma unroll 4
        for (int i = 0; i + 1 < n; ++i) {
          if (fabs(u) <= tiny) u = tiny;
          const double ru = rcp_nr(u);
          su[i * r + l] = ru;  // 1 / u_i for the backward pass
          sy[i * r + l] = y;
          const double lm = s_ea[i] * ru;
          u = s_d[i + 1] - lam - lm * s_ea[i];
          y = sy[(i + 1) * r + l] - lm * y;
        }
        if (fabs(u) <= tiny) u = tiny;
        double xnext = y / u, nrm2 = xnext * xnext;
        sy[(n - 1) * r + l] = xnext;
  #pragma unroll 4
        for (int i = n - 2; i >= 0; --i) {
          const double xi = (sy[i * r + l] - s_ea[i] * xnext) * su[i * r + l];
          sy[i * r + l] = xi;
          nrm2 += xi * xi;
          xnext = xi;
        }
        const double inv = 1.0 / sqrt(nrm2);
        for (int i = 0; i < n; ++i) sy[i * r + l] *= inv;
      }
      // the Rayleigh quotient z^T T_r z of the normalised vector
      double rq = 0.0, zp = 0.0;
      for (int i = 0; i < n; ++i) {
        const double zi = sy[i * r + l];
        rq += zi * (s_d[i] * zi + 2.0 * (i > 0 ? s_ea[i - 1] * zp : 0.0));
        zp = zi;
      }
      s_lam[l] = rq;
    }
    wave_sync();
    // orthogonalise within clusters of close eigenvalues, twice, in descending order
    for (int j = 1; j < r; ++j) {
      bool any = false;
      for (int jp = 0; jp < j; ++jp) any = any || fabs(s_lam[jp] - s_lam[j]) <= 1e-3 * scale;
      if (!any) continue;
      for (int rep = 0; rep < 2; ++rep) {
        for (int jp = 0; jp < j; ++jp) {
          if (!(fabs(s_lam[jp] - s_lam[j]) <= 1e-3 * scale)) continue;
          double dot = 0.0;
          for (int i = l; i < n; i += 64) dot += sy[i * r + jp] * sy[i * r + j];
          dot = wave_sum(dot);
          for (int i = l; i < n; i += 64) sy[i * r + j] -= dot * sy[i * r + jp];
          wave_sync();
        }
      }
      double nn = 0.0;
      for (int i = l; i < n; i += 64) nn += sy[i * r + j] * sy[i * r + j];
      const double inv = 1.0 / sqrt(wave_sum(nn));
      for (int i = l; i < n; i += 64) sy[i * r + j] *= inv;
      wave_sync();
    }
    if (IN_LDS && r <= 8) {  // 5. Y = Q D Z by this wave alone, Y in registers
      if (a.lam_out) {  // only the spectrum was asked for
        if (l < r) a.lam_out[l] = s_lam[l];
        return;
      }
      if (!(s_lam[r - 1] > 1e-14 * s_lam[0]) || !(s_lam[0] > 0.0)) {
        if (l == 0) set_error(a.st, 4, -1);
        return;
      }
      backtransform_wave<8, 8>(Vh, ld, s_beta, s_ph, sy, s_lam, n, r, l, a.Vs);
      return;
    }
    // ---- 5. Y = Q D Z, Y [i * r + j] complex over the start of A's region
    double zr[2][16];
  #pragma unroll
    for (int h = 0; h < 2; ++h)
  #pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = l + 64 * h;
        zr[h][j] = (i < n && j < r) ? sy[i * r + j] : 0.0;
      }
    wave_sync();
    double2* const Y0 = A;
  #pragma unroll
    for (int h = 0; h < 2; ++h)
  #pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = l + 64 * h;
        if (i < n && j < r) Y0[i * r + j] = make_double2(s_ph[i].x * zr[h][j], s_ph[i].y * zr[h][j]);
      }
    wave_sync();
  }
  if (IN_LDS && r <= 8) return;  // every other wave is done after the reduction
  __syncthreads();
  // back-transformation Y <- H_k Y, k descending, over the workgroup (q > 64 or r > 8):
  // thread = (column jc = tid % 16, rows g, g + 64 with g = tid / 16), the same
  // rows for the column sums and the update, so that a thread only reads the
  // rows of Y it wrote; the reflector's values at those rows are loaded one
  // column ahead (they live in global memory for q > 64); column sums by
  // shuffles within a wave, then across the 16 waves through LDS
  double2* Y = A;
  const int jc = tid & 15, g64 = tid >> 4;
  double2* s_sj = &s_p[0][0];  // [wave][16] partial sums, then the 16 totals
  double2 vc[2], vn[2];
  auto vload = [&](int k, double2 (&dst)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) dst[h] = Vh[min(g64 + 64 * h, n - 1) * ld + max(k, 0)];
  };
  vload(n - 3, vc);
  for (int k = n - 3; k >= 0; --k) {
    vload(k - 1, vn);
    const double beta = s_beta[k];
    if (beta != 0.0) {  // the same in every thread
      double2 sj = make_double2(0.0, 0.0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = g64 + 64 * h;
        if (jc < r && i > k && i < n) sj = dadd(sj, djmul(vc[h], Y[i * r + jc]));
      }
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        sj.x += __shfl_xor(sj.x, off);
        sj.y += __shfl_xor(sj.y, off);
      }
      if (l < 16) s_sj[wv * 16 + l] = sj;
      __syncthreads();
      if (tid < 16) {
        double2 t = make_double2(0.0, 0.0);
        for (int w = 0; w < NT / 64; ++w) t = dadd(t, s_sj[w * 16 + tid]);
        s_sj[256 + tid] = make_double2(beta * t.x, beta * t.y);
      }
      __syncthreads();
      // (the next step's totals are written after its first barrier, which
      // every thread reaches only once its update here is done)
      const double2 sv = s_sj[256 + jc];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = g64 + 64 * h;
        if (jc < r && i > k && i < n) Y[i * r + jc] = dsub(Y[i * r + jc], dmul(vc[h], sv));
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) vc[h] = vn[h];
  }
  __syncthreads();  // every row of Y is final before the columns are scaled below
  if (a.lam_out) {  // only the spectrum was asked for
    if (tid < r) a.lam_out[tid] = s_lam[tid];
    return;
  }
  const double lam0 = s_lam[0], lamr = s_lam[r - 1];
  if (!(lamr > 1e-14 * lam0) || !(lam0 > 0.0)) {
    if (tid == 0) set_error(a.st, 4, -1);
    return;
  }
  for (int e2 = tid; e2 < n * r; e2 += NT) {
    const int j = e2 % r;
    const double sc = 1.0 / sqrt(s_lam[j]);
    const double2 v = Y[e2];  // Y[k][j] with e2 = k * r + j
    a.Vs[e2] = make_float2((float)(v.x * sc), (float)(v.y * sc));
  }
}

// U0[:, j] = sum_k X0[:, k] Vs[k][j]: a workgroup takes 64 pixels, its four
// waves the same pixels and a quarter of the r <= RT columns each (the
// frames' values, loaded by each wave, come from the cache for three of
// them); the frames' values KB at a time in flight, every LDS read of Vs
// unconditional (a read under a branch would be waited on alone)
template <int RT>
__global__ __launch_bounds__(AG_NT) void k_x_times_v(const float2* X, const float2* Vs, int n, int q, int r,
                                                     float2* U, const DevState* st) {
  static_assert(AG_NT == 256, "four waves per workgroup");
  constexpr int CPT = RT / 4;  // columns per thread
  __shared__ float2 V[128 * 16];
  const int tid = threadIdx.x, pl = tid & 63, jg = tid >> 6;
  const long p = (long)blockIdx.x * 64 + pl, pc = min(p, (long)n - 1);
  // the first frames' values requested before the state and the table (valid, clamped addresses)
  constexpr int KB = 16;
  float2 xv[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) xv[i] = X[(long)min(i, q - 1) * n + pc];
  if (st->err) return;
  for (int e = tid; e < q * r; e += AG_NT) V[e] = Vs[e];
  __syncthreads();
  int jc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) jc[c] = min(jg * CPT + c, r - 1);
  float2 acc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) acc[c] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < q; k0 += KB) {
    float2 xn[KB];
    const bool more = k0 + KB < q;
#pragma unroll
    for (int i = 0; i < KB; ++i) xn[i] = X[(long)min(k0 + KB + i, q - 1) * n + pc];  // the next batch
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const int k = min(k0 + i, q - 1);
      const float2 x = (k0 + i < q) ? xv[i] : make_float2(0.f, 0.f);
      const float2* vk = V + k * r;
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[c] = cadd(acc[c], cmul(x, vk[jc[c]]));
    }
    if (!more) break;
#pragma unroll
    for (int i = 0; i < KB; ++i) xv[i] = xn[i];
  }
  if (p >= n) return;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = jg * CPT + c;
    if (j < r) U[(long)j * n + p] = acc[c];
  }
}

hipError_t launch_x_times_v(const float2* X, const float2* Vs, int n, int q, int r, float2* U, const DevState* st,
                            hipStream_t s) {
  const dim3 g((n + 63) / 64), b(AG_NT);
  if (r <= 8) hipLaunchKernelGGL(k_x_times_v<8>, g, b, 0, s, X, Vs, n, q, r, U, st);
  else hipLaunchKernelGGL(k_x_times_v<16>, g, b, 0, s, X, Vs, n, q, r, U, st);
  return hipGetLastError();
}

// keep the learned U (src) only if its cost f[1] is strictly below the
// spectral one f[0]; a non-finite learned cost keeps the spectral U
// The error and halt flags as they stood before the learned guess was scored
// (raising an error also halts the loop).
__global__ void k_err_snapshot(const DevState* st, int32_t* snap) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    snap[0] = st->err;
    snap[1] = st->halt;
  }
}

// Keep the learned basis (src) only if its cost f[1] is strictly below the
// fallback's f[0].  A guess whose scoring raised an error (a Gram of the
// guess or of A_k U that is not positive definite, a non-finite value) counts
// as infinitely costly: the fallback stays.  An error that was already set
// before the guess was scored (snap) is left for the caller.
__global__ void k_pick_init(const double* f, const int32_t* snap, const float2* src, float2* dst, long n,
                            int32_t* choice, const DevState* st) {
  if (*snap) return;
  const bool take = st->err == 0 && f[1] < f[0];
  if (choice && blockIdx.x == 0 && threadIdx.x == 0) *choice = take ? 1 : 0;
  if (!take) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) dst[i] = src[i];
}

// After k_pick_init: an error raised only by the rejected guess is cleared,
// with the halt it raised.
__global__ void k_err_restore(const int32_t* snap, DevState* st) {
  if (threadIdx.x != 0 || snap[0]) return;
  if (st->err) {
    st->err = 0;
    st->err_frame = -1;
    st->halt = snap[1];
  }
}

__global__ void k_copy(const float2* src, float2* dst, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long stride = (long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_cost_total(const double* cost_k, int q, double* out, DevState* st) {
  if (threadIdx.x != 0) return;
  double f = 0.0;
  for (int k = 0; k < q; ++k) f += cost_k[k];
  st->cost_out = f;
  if (out) *out = f;
}

// ---------------------------------------------------------------------------
// launchers (explicit instantiations behind plain functions)
// ---------------------------------------------------------------------------
hipError_t launch_gram_cols(const GramColsArgs& a, int nblk, bool fp64, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_gram_cols<double>, dim3(nblk), dim3(GCOLS_NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_gram_cols<float>, dim3(nblk), dim3(GCOLS_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply(const ApplyArgs& a, hipStream_t s) {
  const dim3 g((unsigned)((a.n + AG_NT - 1) / AG_NT));
  if (a.r <= 4) hipLaunchKernelGGL(k_apply<4>, g, dim3(AG_NT), 0, s, a);
  else if (a.r <= 8) hipLaunchKernelGGL(k_apply<8>, g, dim3(AG_NT), 0, s, a);
  else if (a.r <= 12) hipLaunchKernelGGL(k_apply<12>, g, dim3(AG_NT), 0, s, a);
  else hipLaunchKernelGGL(k_apply<16>, g, dim3(AG_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qr_small(const QrSmallArgs& a, hipStream_t s) {
  // 1,024 threads for the partial sums at the start; the one-wave factor's
  // rows padded to 8, 12 or 16 with the identity
  if (a.r <= 8) hipLaunchKernelGGL(k_qr_small<8>, dim3(1), dim3(1024), 0, s, a);
  else if (a.r <= 12) hipLaunchKernelGGL(k_qr_small<12>, dim3(1), dim3(1024), 0, s, a);
  else hipLaunchKernelGGL(k_qr_small<16>, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_eig(const InitEigArgs& a, hipStream_t s) {
  if (a.q > 128 || a.r > 16 || a.r > a.q) return hipErrorInvalidValue;
  // q <= 64: matrix and reflectors in LDS; else the packed lower triangle
  // (the reflectors in a.V)
  const size_t lds = a.in_lds ? 2 * (size_t)a.q * (a.q | 1) * sizeof(double2)
                              : (size_t)a.q * (a.q + 1) / 2 * sizeof(double2);
  const void* fn = a.in_lds ? (const void*)k_init_eig<true> : (const void*)k_init_eig<false>;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.in_lds) hipLaunchKernelGGL((k_init_eig<true>), dim3(1), dim3(1024), lds, s, a);
  else hipLaunchKernelGGL((k_init_eig<false>), dim3(1), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace ag
