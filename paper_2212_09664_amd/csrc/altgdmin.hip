// Host side of the C ABI declared in include/altgdmin.h: argument checks,
// workspace carving and the launch sequences of setup, spectral
// initialisation, the altGDmin iteration (Algorithm 2) and the operators.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "ctx.hpp"

using ag_host::map_hip;

namespace {

const char* kTimedNames[TK_COUNT] = {"none",  "fwd_transform", "gram_rhs", "solve",     "fold",
                                     "adj_transform", "qr_gram", "qr_small", "apply_qr"};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace


namespace {


// sum over lines of ceil(pairs / 8) <= (pairs + 7 lines) / 8, pairs <= q * width
// workgroups of the spectral init's X0^H X0 on the matrix cores: 128 rows each, at most 512
int init_nblk(const altgdmin_ctx* c) { return (int)std::max(1L, std::min(512L, ((long)c->n + 127) / 128)); }

long gram_items_bound(const altgdmin_ctx* c) {
  return ((long)c->p.q * c->width + 7L * c->n_loc) / 8 + 1;
}

void carve(altgdmin_ctx* c) {
  const altgdmin_params& p = c->p;
  const int r = p.r, q = p.q, nc = p.nc;
  const long n = c->n;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align256(off + b);
    return o;
  };
  c->o_st = take(sizeof(DevState));
  c->o_twx = take(sizeof(float2) * p.nx);
  c->o_twy = take(sizeof(float2) * p.ny);
  c->o_bitmap = take(sizeof(uint32_t) * (size_t)c->n_loc * c->nw);
  c->o_locptr = take(sizeof(int32_t) * (size_t)(c->n_loc + 1));
  c->o_loc2unit = take(sizeof(int32_t) * (size_t)c->n_loc);
  c->o_unitloc = take(sizeof(int32_t) * (size_t)c->n_loc);
  c->o_unitspan = take(sizeof(int2) * (size_t)c->n_loc);
  c->o_bcp = take(sizeof(float2) * (size_t)q * c->width * r);
  c->o_Uc = take(sizeof(float2) * (size_t)n * r);
  c->o_fcmp = take(sizeof(double) * 4);  // the two costs compared, then the error snapshot
  // Gram work list: at most ceil(q/8) items per line, and at least one entry per
  // workgroup of the Gram launch (ny + 64 of them)
  c->o_gwork = take(sizeof(int4) * ((size_t)c->n_loc * ((q + 7) / 8) + (c->lines ? p.ny + 64 : 0)));
  c->o_lineord = take(sizeof(int4) * (size_t)c->n_loc);  // the fold's line order, most pairs first
  c->o_planes = take(sizeof(double) * 256);
  c->o_coilb = take(sizeof(float2) * (size_t)n * nc);
  c->o_yg = take(c->lines ? sizeof(float2) * 8 * (size_t)gram_items_bound(c) * nc * p.nx : 0);
  c->o_pairs = take(sizeof(int2) * (size_t)q * c->width);
  c->o_pairof = take(sizeof(int32_t) * (size_t)q * c->width);
  c->o_unitof = take(sizeof(int32_t) * (size_t)q * c->width);
  c->o_Ui = take(sizeof(float2) * (size_t)n * r);
  const size_t ysz = sizeof(float2) * (size_t)q * nc * p.m_max;
  c->o_yh = take(c->lines ? ysz : 0);
  c->o_ysq = take(sizeof(double) * q);
  c->o_ysqp = take(sizeof(double) * q * nc);
  c->o_cost = take(sizeof(double) * q);
  const size_t wsz = sizeof(float2) * (size_t)nc * r * c->ua * p.nx;
  c->o_W = take(wsz);
  c->o_K = take(wsz);
  const int nP = r * (r + 1) / 2;
  if (c->lines) {
    c->o_P = take(sizeof(double2) * (size_t)c->gram_ngroups * p.ny * r * r);
    c->o_hp = take(sizeof(double2) * (size_t)c->gram_ngroups * q * c->width * r);
  } else {
    c->o_P = take(sizeof(double2) * (size_t)q * c->nchunks * nc * (r * r + r));
    c->o_hp = take(0);
  }
  c->o_B = take(sizeof(float2) * (size_t)q * r);
  c->o_G = take(sizeof(float2) * (size_t)c->adj_parts * n * r);
  const int m_iter = 2 * r;
  const size_t qo = (size_t)std::max(m_iter * (m_iter + 1) / 2, q * (q + 1) / 2);
  // QR Gram partials; the spectral init's Gram uses up to init_nblk of them
  // plus one slot for their sum
  c->o_qpart = take(sizeof(double2) * qo * (std::max(std::max(c->qr_nblk, init_nblk(c)), p.nx) + 1));
  c->o_qtot = take(sizeof(double2) * m_iter * (m_iter + 1) / 2);  // their sum (the fused step)
  c->o_rfac = take(sizeof(float2) * r * r);
  c->o_stsrc = take(sizeof(double2) * 193);  // deferred statistics of the fused step
  c->o_Vs = take(sizeof(float2) * (size_t)q * r);
  c->o_V = take(sizeof(double2) * 2 * (size_t)q * (q | 1));  // matrix and reflectors, odd row pitch
  // temp: X0 plus the truncated hybrid data (LINES) or a chunk of coil images (INDEX)
  size_t tb = sizeof(float2) * (size_t)n * q;
  if (c->lines)
    tb += ysz;
  else
    tb += sizeof(float2) * (size_t)c->kc * nc * n;
  c->T_bytes = tb;
  c->o_T = take(tb);
  c->o_end = off;
  c->bytes = off;
}

altgdmin_status check_params(const altgdmin_params* p) {
  if (!p) return ALTGDMIN_EINVAL;
  if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < 8 || p->ny < 8 || p->nx > 512 || p->ny > 512)
    return ALTGDMIN_EINVAL;
  if (p->nc < 1 || p->nc > 64 || p->q < 1 || p->q > 128 || p->r < 1 || p->r > 16)
    return ALTGDMIN_EINVAL;
  if (p->mask_kind != ALTGDMIN_MASK_LINES && p->mask_kind != ALTGDMIN_MASK_INDEX) return ALTGDMIN_EINVAL;
  if (p->precision != ALTGDMIN_FP32 && p->precision != ALTGDMIN_MIXED) return ALTGDMIN_EINVAL;
  if (p->m_max < 1 || p->m_max > p->nx * p->ny) return ALTGDMIN_EINVAL;
  if (p->mask_kind == ALTGDMIN_MASK_LINES && (p->m_max % p->nx) != 0) return ALTGDMIN_EINVAL;
  if (!(p->eta_c > 0) || !isfinite(p->eta_c) || !isfinite(p->trunc_c) || !(p->eta_cap_c >= 0) ||
      !isfinite(p->eps_exit) || p->exit_consec < 0)
    return ALTGDMIN_EINVAL;
  if (p->t_max < 1) return ALTGDMIN_EINVAL;
  return ALTGDMIN_OK;
}

// ---- timing of one kernel class ------------------------------------------
void tmark(altgdmin_ctx* c, int which) {
  if (c->timed != which) return;
  if (c->ev_used + 1 >= c->ev.size()) {
    for (int i = 0; i < 256; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->ev.push_back(e);
    }
  }
  (void)hipEventRecord(c->ev[c->ev_used++], c->stream);
}

// ---- launch sequences -------------------------------------------------------
BasisArgs basis_args(altgdmin_ctx* c, int check_halt) {
  const altgdmin_params& p = c->p;
  BasisArgs b{};
  b.U = c->at<float2>(c->o_Ui);
  b.W = c->at<float2>(c->o_W);
  b.K = c->at<float2>(c->o_K);
  b.G = c->at<float2>(c->o_G);
  b.coils = c->at<float2>(c->o_coilb);
  b.n = c->n;
  b.nx = p.nx;
  b.r = p.r;
  b.nc = p.nc;
  b.ua = c->ua;
  b.txx = c->txx;
  b.cgs = c->adj_cgs;
  b.part_stride = (long)c->n * p.r;
  if (c->lines) {
    b.rows = c->at<int32_t>(c->o_unitloc);
    b.n_rows_ptr = &c->st()->n_units;
    b.row_unit = c->at<int32_t>(c->o_loc2unit);
  }
  b.tw = c->at<float2>(c->o_twy);
  b.tw_x = c->at<float2>(c->o_twx);
  b.scale = (float)(1.0 / sqrt((double)p.ny));
  b.scale_x = (float)(1.0 / sqrt((double)p.nx));
  b.st = c->st();
  b.check_halt = check_halt;
  return b;
}

// the pixel-major working copy of a column-major basis
hipError_t to_pixmajor(altgdmin_ctx* c, const float2* U) {
  hipLaunchKernelGGL(k_to_pixmajor, dim3(512), dim3(256), 0, c->stream, U, c->p.r, (long)c->n,
                     c->at<float2>(c->o_Ui));
  return hipGetLastError();
}

PdftArgs pdft_args(altgdmin_ctx* c, int check_halt) {
  const altgdmin_params& p = c->p;
  PdftArgs a{};
  a.U = c->at<float2>(c->o_Ui);
  a.coils = c->coils;
  a.W = c->at<float2>(c->o_W);
  a.K = c->at<float2>(c->o_K);
  a.G = c->at<float2>(c->o_G);
  a.tw = c->at<float2>(c->o_twy);
  a.unit_loc = c->at<int32_t>(c->o_unitloc);
  a.nx = p.nx;
  a.r = p.r;
  a.nc = p.nc;
  a.ua = c->ua;
  a.cgs = c->adj_cgs;
  a.n = c->n;
  a.part_stride = (long)c->n * p.r;
  a.scale = (float)(1.0 / sqrt((double)p.ny));
  a.st = c->st();
  a.check_halt = check_halt;
  return a;
}

// W_{c,j} = F(s_c o u_j) on the sampled rows (y half only for LINES), from
// the pixel-major working copy of U
hipError_t fwd_transform(altgdmin_ctx* c, int check_halt) {
  const altgdmin_params& p = c->p;
  if (c->pdft)
    return launch_pdft(0, p.ny, pdft_args(c, check_halt), (p.nx * p.r + 31) / 32,
                       p.ny == 256 ? c->adj_parts : p.nc, c->stream);  // coil groups in the factored form
  const BasisArgs b = basis_args(c, check_halt);
  hipError_t e = launch_basis(0, p.ny, b, p.nx / c->txx, c->adj_parts, c->stream);
  if (e != hipSuccess || c->lines) return e;
  return launch_basis(2, p.nx, b, p.nc * p.ny, 1, c->stream);
}

hipError_t gram_solve(altgdmin_ctx* c, int check_halt) {
  const altgdmin_params& p = c->p;
  hipError_t e;
  if (c->lines) {
    GramLinesArgs g{};
    g.W = c->at<float2>(c->o_W);
    g.yu = c->at<float2>(c->o_yh);
    g.yg = c->at<float2>(c->o_yg);
    g.items = c->at<int4>(c->o_gwork);
    g.pairs = c->at<int2>(c->o_pairs);
    g.loc_ptr = c->at<int32_t>(c->o_locptr);
    g.unit_loc = c->at<int32_t>(c->o_unitloc);
    g.nc = p.nc;
    g.r = p.r;
    g.nx = p.nx;
    g.ua = c->ua;
    g.cg = c->gram_cg;
    g.npairs = (long)p.q * c->width;
    g.P = c->at<double2>(c->o_P);
    g.hp = c->at<double2>(c->o_hp);
    g.st = c->st();
    g.check_halt = check_halt;
    tmark(c, TK_GRAM);
    e = launch_gram_lines(g, p.ny, c->gram_ngroups, p.q, c->fp64, c->stream);
    tmark(c, TK_GRAM);
  } else {
    GramIndexArgs g{};
    g.W = c->at<float2>(c->o_W);
    g.y = c->y;
    g.mask = c->mask;
    g.m_k = c->m_k;
    g.nc = p.nc;
    g.r = p.r;
    g.n = c->n;
    g.m_max = p.m_max;
    g.chunk = c->gram_chunk;
    g.nchunks = c->nchunks;
    g.part = c->at<double2>(c->o_P);
    g.st = c->st();
    g.check_halt = check_halt;
    tmark(c, TK_GRAM);
    e = launch_gram_index(g, p.q, c->fp64, c->stream);
    tmark(c, TK_GRAM);
  }
  if (e != hipSuccess) return e;
  SolveArgs s{};
  s.P = c->at<double2>(c->o_P);
  s.hp = c->at<double2>(c->o_hp);
  s.mask = c->mask;
  s.m_k = c->m_k;
  s.pair_of = c->at<int32_t>(c->o_pairof);
  s.unit_of = c->at<int32_t>(c->o_unitof);
  s.width = c->width;
  s.nx = p.nx;
  s.r = p.r;
  s.kind = c->lines ? 0 : 1;
  s.nchunks = c->nchunks * p.nc;  // INDEX: partials per frame, one per (chunk, coil)
  s.ngroups = c->gram_ngroups;
  s.ua = c->ua;
  s.npairs = (long)p.q * c->width;
  s.ysq_k = c->at<double>(c->o_ysq);
  s.B = c->at<float2>(c->o_B);
  s.B_out = c->b_out;
  s.bcp = c->at<float2>(c->o_bcp);
  s.cost_k = c->at<double>(c->o_cost);
  s.st = c->st();
  s.check_halt = check_halt;
  tmark(c, TK_SOLVE);
  e = launch_solve(s, p.q, c->fp64, c->stream);
  tmark(c, TK_SOLVE);
  return e;
}

hipError_t cholqr(altgdmin_ctx* c, float2* U) {
  const altgdmin_params& p = c->p;
  hipError_t e0 = to_pixmajor(c, U);
  if (e0 != hipSuccess) return e0;
  GramColsArgs g{};
  g.A = c->at<float2>(c->o_Ui);
  g.m1 = p.r;
  g.m2 = 0;
  g.n = c->n;
  g.rows_per_block = c->qr_rows;
  g.nparts = 1;
  g.part = c->at<double2>(c->o_qpart);
  g.st = c->st();
  hipError_t e = launch_qr_gram(g, c->qr_nblk, true, c->stream);
  if (e != hipSuccess) return e;
  QrSmallArgs qa{};
  qa.part = c->at<double2>(c->o_qpart);
  qa.nblk = c->qr_nblk;
  qa.r = p.r;
  qa.mode = 1;
  qa.n = c->n;
  qa.q = p.q;
  qa.rfac = c->at<float2>(c->o_rfac);
  qa.st = c->st();
  e = launch_qr_small(qa, c->stream);
  if (e != hipSuccess) return e;
  ApplyArgs aa{};
  aa.U = U;
  aa.Ui = c->at<float2>(c->o_Ui);
  aa.rfac = c->at<float2>(c->o_rfac);
  aa.n = c->n;
  aa.r = p.r;
  aa.mode = 1;
  aa.st = c->st();
  return launch_apply(aa, c->stream);
}

// b_k for every frame and the gradient at U (into the workspace's B and G)
hipError_t gradient_pieces(altgdmin_ctx* c, int check_halt) {
  const altgdmin_params& p = c->p;
  hipError_t e;
  tmark(c, TK_FWD);
  e = fwd_transform(c, check_halt);
  tmark(c, TK_FWD);
  if (e != hipSuccess) return e;
  e = gram_solve(c, check_halt);
  if (e != hipSuccess) return e;
  // fold the residual over frames
  FoldArgs fa{};
  fa.line_order = c->at<int4>(c->o_lineord);
  fa.bcp = c->at<float2>(c->o_bcp);
  fa.W = c->at<float2>(c->o_W);
  fa.yu = c->at<float2>(c->o_yh);
  fa.y = c->y;
  fa.B = c->at<float2>(c->o_B);
  fa.pairs = c->at<int2>(c->o_pairs);
  fa.loc_ptr = c->at<int32_t>(c->o_locptr);
  fa.nc = p.nc;
  fa.r = p.r;
  fa.nx = p.nx;
  fa.ua = c->ua;
  fa.n = c->n;
  fa.m_max = p.m_max;
  fa.max_pairs = p.q;
  fa.K = c->at<float2>(c->o_K);
  fa.st = c->st();
  fa.check_halt = check_halt;
  tmark(c, TK_FOLD);
  if (c->lines) {
    e = launch_fold2(fa, true, p.nc, p.ny, c->stream);
  } else {
    e = launch_fold2(fa, false, 0, p.nc, c->stream);  // the launcher sizes the grid
  }
  tmark(c, TK_FOLD);
  if (e != hipSuccess) return e;
  // inverse transform + coil combine -> partial gradients per coil group
  tmark(c, TK_ADJ);
  if (c->pdft) {
    e = launch_pdft(1, p.ny, pdft_args(c, check_halt), (p.nx * p.r + 31) / 32, c->adj_parts, c->stream);
    tmark(c, TK_ADJ);
    return e;
  }
  const BasisArgs b = basis_args(c, check_halt);
  if (!c->lines) {
    e = launch_basis(3, p.nx, b, p.nc * p.ny, 1, c->stream);
    if (e != hipSuccess) return e;
  }
  if (c->adj_qr) {
    BasisArgs bq = b;
    bq.qpart = reinterpret_cast<float2*>(c->at<double2>(c->o_qpart));
    e = launch_adj_qr(p.ny, bq, c->stream);
  } else {
    e = launch_basis(1, p.ny, b, p.nx / c->txx, c->adj_parts, c->stream);
  }
  tmark(c, TK_ADJ);
  return e;
}

// Gram of [U grad] (summing the partial gradients) and the small QR-step
// work; mode 0 a step, mode 2 only the step size at the first iteration
// the QR Gram of [U grad] (summing the adjoint's partial gradients)
hipError_t qr_step_gram(altgdmin_ctx* c, int check_halt) {
  if (c->adj_qr) return hipSuccess;  // the adjoint transform wrote the block partials
  const altgdmin_params& p = c->p;
  GramColsArgs g{};
  g.A = c->at<float2>(c->o_Ui);
  g.B = c->at<float2>(c->o_G);
  g.m1 = p.r;
  g.m2 = p.r;
  g.n = c->n;
  g.rows_per_block = c->qr_rows;
  g.nparts = c->grad_parts;
  g.part_stride = (long)c->n * p.r;
  g.write_sum = 1;
  g.part = c->at<double2>(c->o_qpart);
  g.st = c->st();
  g.check_halt = check_halt;
  tmark(c, TK_QRGRAM);
  hipError_t e = launch_qr_gram(g, c->qr_nblk, c->fp64, c->stream);
  tmark(c, TK_QRGRAM);
  return e;
}

QrSmallArgs qr_small_args(altgdmin_ctx* c, int mode, int check_halt) {
  const altgdmin_params& p = c->p;
  QrSmallArgs qa{};
  qa.part = c->at<double2>(c->o_qpart);
  qa.part_f32 = !c->fp64;
  qa.nblk = c->adj_qr ? p.nx : c->qr_nblk;  // one block per image column, or per row block
  qa.r = p.r;
  qa.mode = mode;
  qa.n = c->n;
  qa.q = p.q;
  qa.eta_c = p.eta_c;
  qa.eta_cap_c = p.eta_cap_c;
  qa.eps_exit = p.eps_exit;
  qa.exit_consec = p.exit_consec > 1 ? p.exit_consec : 1;
  qa.guard = 1e-6;  // FP32 gradient: below this it is rounding noise
  qa.B = c->at<float2>(c->o_B);
  qa.cost_k = c->at<double>(c->o_cost);
  qa.rfac = c->at<float2>(c->o_rfac);
  qa.st = c->st();
  qa.check_halt = check_halt;
  return qa;
}

hipError_t qr_step_small(altgdmin_ctx* c, int mode, int check_halt) {
  hipError_t e = qr_step_gram(c, check_halt);
  if (e != hipSuccess) return e;
  const QrSmallArgs qa = qr_small_args(c, mode, check_halt);
  tmark(c, TK_QRSMALL);
  e = launch_qr_small(qa, c->stream);
  tmark(c, TK_QRSMALL);
  return e;
}

// the step and the update fused (rank <= 8): QR Gram, then one kernel that
// factors and updates, then (exit rule on) the commit of its outcome
hipError_t qr_step_apply(altgdmin_ctx* c, float2* U, float2* U_prev) {
  const altgdmin_params& p = c->p;
  hipError_t e = qr_step_gram(c, 1);
  if (e != hipSuccess) return e;
  QrSmallArgs qa = qr_small_args(c, 0, 1);
  tmark(c, TK_APPLY);
  const int nout = p.r * (2 * p.r + 1);
  e = launch_partials_total(qa.part, qa.part_f32, qa.nblk, nout, c->at<double2>(c->o_qtot), c->stream);
  if (e != hipSuccess) return e;
  qa.part = c->at<double2>(c->o_qtot);  // the partials summed (FP64)
  qa.part_f32 = 0;
  qa.nblk = 1;
  qa.commit_direct = !(p.eps_exit > 0.0);
  qa.stats_src = c->at<double2>(c->o_stsrc);
  ApplyArgs aa{};
  aa.U = U;
  aa.Ui = c->at<float2>(c->o_Ui);
  aa.G = c->at<float2>(c->o_G);
  aa.rfac = c->at<float2>(c->o_rfac);
  aa.U_prev = U_prev;
  aa.n = c->n;
  aa.r = p.r;
  aa.mode = 0;
  aa.st = c->st();
  e = launch_step_apply(qa, aa, c->stream);
  tmark(c, TK_APPLY);
  return e;
}

hipError_t one_iteration(altgdmin_ctx* c, float2* U, float2* U_prev) {
  const altgdmin_params& p = c->p;
  hipError_t e = gradient_pieces(c, 1);
  if (e != hipSuccess) return e;
  if (p.r <= 8) return qr_step_apply(c, U, U_prev);
  e = qr_step_small(c, 0, 1);
  if (e != hipSuccess) return e;
  ApplyArgs aa{};
  aa.U = U;
  aa.Ui = c->at<float2>(c->o_Ui);
  aa.G = c->at<float2>(c->o_G);
  aa.rfac = c->at<float2>(c->o_rfac);
  aa.U_prev = U_prev;
  aa.n = c->n;
  aa.r = p.r;
  aa.mode = 0;
  aa.st = c->st();
  tmark(c, TK_APPLY);
  e = launch_apply(aa, c->stream);
  tmark(c, TK_APPLY);
  return e;
}

}  // namespace

#define AGCHK(x)                           \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) return _e;       \
  } while (0)

namespace ag_host {

// X = A^H(Y) scaled per column (back-projection when trunc/scale are set)
hipError_t adjoint_op(altgdmin_ctx* c, const float2* Y, float2* X, int trunc, int scale_mk) {
  const altgdmin_params& p = c->p;
  hipError_t e;
  float2* T = c->at<float2>(c->o_T) + (size_t)c->n * p.q;  // after the X0 slot
  if (c->lines) {
    RowArgs ra{};
    ra.src = Y;
    ra.dst = T;
    ra.tw = c->at<float2>(c->o_twx);
    ra.nrows = (long)p.q * p.nc * c->lmax;
    ra.m_k = c->m_k;
    ra.nc = p.nc;
    ra.lmax = c->lmax;
    ra.scale = (float)(1.0 / sqrt((double)p.nx));
    ra.trunc = trunc;
    ra.trunc_count = trunc ? &c->st()->n_trunc : nullptr;
    ra.st = c->st();
    e = launch_rows(p.nx, ra, true, c->stream);
    if (e != hipSuccess) return e;
    ColAdjArgs d{};
    d.src = T;
    d.src_c_stride = (long)c->lmax * p.nx;
    d.src_img_stride = (long)p.nc * c->lmax * p.nx;
    d.rows = c->mask;
    d.rows_img_stride = c->width;
    d.m_k_rows = c->m_k;
    d.coils = c->coils;
    d.n = c->n;
    d.nx = p.nx;
    d.nc = p.nc;
    d.tw = c->at<float2>(c->o_twy);
    d.dst = X;
    d.dst_img_stride = c->n;
    d.m_k_scale = scale_mk ? c->m_k : nullptr;
    d.scale = (float)(1.0 / sqrt((double)p.ny));
    d.st = c->st();
    return launch_cols(p.ny, nullptr, &d, p.nx, p.q, p.nc, c->stream);
  }
  for (int k0 = 0; k0 < p.q; k0 += c->kc) {
    const int kc = std::min(c->kc, p.q - k0);
    const long nimg = (long)kc * p.nc * c->n;
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, c->stream, T, nimg);
    hipLaunchKernelGGL(k_scatter, dim3((p.m_max + 255) / 256, kc, p.nc), dim3(256), 0, c->stream, Y, c->mask,
                       c->m_k, p.m_max, p.nc, k0, T, (long)c->n, (long)p.nc * c->n, c->st(), trunc,
                       trunc ? &c->st()->n_trunc : nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    RowArgs ra{};
    ra.src = ra.dst = T;
    ra.tw = c->at<float2>(c->o_twx);
    ra.nrows = (long)kc * p.nc * p.ny;
    ra.scale = (float)(1.0 / sqrt((double)p.nx));
    ra.st = c->st();
    e = launch_rows(p.nx, ra, true, c->stream);
    if (e != hipSuccess) return e;
    ColAdjArgs d{};
    d.src = T;
    d.src_c_stride = c->n;
    d.src_img_stride = (long)p.nc * c->n;
    d.coils = c->coils;
    d.n = c->n;
    d.nx = p.nx;
    d.nc = p.nc;
    d.tw = c->at<float2>(c->o_twy);
    d.dst = X + (size_t)k0 * c->n;
    d.dst_img_stride = c->n;
    d.m_k_scale = scale_mk ? c->m_k + k0 : nullptr;
    d.scale = (float)(1.0 / sqrt((double)p.ny));
    d.st = c->st();
    e = launch_cols(p.ny, nullptr, &d, p.nx, kc, p.nc, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}



hipError_t forward_op(altgdmin_ctx* c, const float2* X, float2* Y) {
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  if (c->lines) {
    ColFwdArgs f{};
    f.src = X;
    f.src_img_stride = c->n;
    f.coils = c->coils;
    f.n = c->n;
    f.nx = p.nx;
    f.tw = c->at<float2>(c->o_twy);
    f.dst = Y;
    f.dst_c_stride = p.m_max;
    f.dst_img_stride = (long)p.nc * p.m_max;
    f.rows = c->mask;
    f.rows_img_stride = c->width;
    f.m_k = c->m_k;
    f.zero_pad_rows = c->lmax;
    f.scale = (float)(1.0 / sqrt((double)p.ny));
    f.st = c->st();
    AGCHK(launch_cols(p.ny, &f, nullptr, p.nx, p.q, p.nc, s));
    RowArgs ra{};
    ra.src = ra.dst = Y;
    ra.tw = c->at<float2>(c->o_twx);
    ra.nrows = (long)p.q * p.nc * c->lmax;
    ra.m_k = c->m_k;
    ra.nc = p.nc;
    ra.lmax = c->lmax;
    ra.scale = (float)(1.0 / sqrt((double)p.nx));
    ra.st = c->st();
    AGCHK(launch_rows(p.nx, ra, false, s));
    return hipSuccess;
  }
  float2* T = c->at<float2>(c->o_T) + (size_t)c->n * p.q;
  for (int k0 = 0; k0 < p.q; k0 += c->kc) {
    const int kc = std::min(c->kc, p.q - k0);
    ColFwdArgs f{};
    f.src = X + (size_t)k0 * c->n;
    f.src_img_stride = c->n;
    f.coils = c->coils;
    f.n = c->n;
    f.nx = p.nx;
    f.tw = c->at<float2>(c->o_twy);
    f.dst = T;
    f.dst_c_stride = c->n;
    f.dst_img_stride = (long)p.nc * c->n;
    f.scale = (float)(1.0 / sqrt((double)p.ny));
    f.st = c->st();
    AGCHK(launch_cols(p.ny, &f, nullptr, p.nx, kc, p.nc, s));
    RowArgs ra{};
    ra.src = ra.dst = T;
    ra.tw = c->at<float2>(c->o_twx);
    ra.nrows = (long)kc * p.nc * p.ny;
    ra.scale = (float)(1.0 / sqrt((double)p.nx));
    ra.st = c->st();
    AGCHK(launch_rows(p.nx, ra, false, s));
    hipLaunchKernelGGL(k_gather, dim3((p.m_max + 255) / 256, kc, p.nc), dim3(256), 0, s, T, (long)c->n,
                       (long)p.nc * c->n, c->mask, c->m_k, p.m_max, p.nc, k0, Y, c->st());
    AGCHK(hipGetLastError());
  }
  return hipSuccess;
}


hipError_t spectral_eig(altgdmin_ctx* c, int r_eig, double* lam_out) {
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  float2* X0 = c->at<float2>(c->o_T);
  AGCHK(adjoint_op(c, c->y, X0, p.trunc_c > 0 ? 1 : 0, 1));
  GramColsArgs g{};
  g.A = X0;
  g.m1 = p.q;
  g.m2 = 0;
  g.n = c->n;
  g.rows_per_block = c->qr_rows;
  g.part = c->at<double2>(c->o_qpart);
  g.st = c->st();
  g.nparts = 1;
  g.a_colmajor = 1;
  // X0^H X0 in FP64 on the matrix cores (f64 16x16x4) over many short
  // workgroups (k_init_gram up to 48 frames, k_init_gram_cx up to 128), whose
  // partials a second kernel sums
  InitEigArgs ie{};
  if (p.q <= 128) {
    const int nb = init_nblk(c);
    g.rows_per_block = ((c->n + nb - 1) / nb + 31) / 32 * 32;
    const int nbu = (int)((c->n + g.rows_per_block - 1) / g.rows_per_block);
    if (p.q <= 48) AGCHK(launch_init_gram(g, nbu, s));
    else AGCHK(launch_init_gram_cx(g, nbu, s));
    const int nout = p.q * (p.q + 1) / 2;
    double2* sum = c->at<double2>(c->o_qpart) + (size_t)nbu * nout;
    AGCHK(launch_sum_partials(c->at<double2>(c->o_qpart), nbu, nout, sum, s));
    ie.part = sum;
    ie.nblk = 1;
  } else {
    AGCHK(launch_gram_cols(g, c->qr_nblk, true, s));
    ie.part = c->at<double2>(c->o_qpart);
    ie.nblk = c->qr_nblk;
  }
  ie.q = p.q;
  ie.r = r_eig;
  ie.lam_out = lam_out;
  ie.V = c->at<double2>(c->o_V);
  ie.in_lds = p.q <= 64;
  ie.Vs = c->at<float2>(c->o_Vs);
  ie.st = c->st();
  AGCHK(launch_init_eig(ie, s));
  return hipSuccess;
}

}  // namespace ag_host

extern "C" {

const char* altgdmin_status_string(altgdmin_status s) {
  switch (s) {
    case ALTGDMIN_OK: return "ok";
    case ALTGDMIN_EINVAL: return "invalid argument";
    case ALTGDMIN_ESTATE: return "call out of order";
    case ALTGDMIN_EHIP: return "HIP runtime error";
    case ALTGDMIN_ENOTPD: return "Gram matrix not positive definite";
    case ALTGDMIN_ENONFINITE: return "non-finite value";
    case ALTGDMIN_EUNSUPPORTED: return "unsupported configuration";
    case ALTGDMIN_ESCRATCH: return "problem too large for the built-in scratch";
  }
  return "unknown status";
}

altgdmin_status altgdmin_create(const altgdmin_params* params, altgdmin_ctx** out) {
  if (!out) return ALTGDMIN_EINVAL;
  *out = nullptr;
  altgdmin_status s = check_params(params);
  if (s != ALTGDMIN_OK) return s;
  altgdmin_ctx* c = new (std::nothrow) altgdmin_ctx();
  if (!c) return ALTGDMIN_EINVAL;
  c->p = *params;
  const altgdmin_params& p = c->p;
  c->n = p.nx * p.ny;
  c->lines = (p.mask_kind == ALTGDMIN_MASK_LINES);
  c->fp64 = (p.precision == ALTGDMIN_MIXED);
  c->pdft = c->fp64 && p.mask_kind == ALTGDMIN_MASK_LINES && p.ny >= 32 && p.ny <= 256;
  c->lmax = c->lines ? p.m_max / p.nx : 0;
  c->width = c->lines ? c->lmax : p.m_max;
  c->per = c->lines ? p.nx : 1;
  c->n_loc = c->lines ? p.ny : c->n;
  c->nw = (p.q + 31) / 32;
  c->ua = p.ny;
  c->gram_chunk = GRAM_INDEX_CHUNK;
  c->nchunks = (p.m_max + c->gram_chunk - 1) / c->gram_chunk;
  c->gram_cg = std::max(1, std::min(p.nc, 1024 / p.nx));
  c->gram_ngroups = (p.nc + c->gram_cg - 1) / c->gram_cg;
  c->txx = basis_txx(p.ny, p.nx, p.r);
  {
    const int tiles = p.nx / c->txx;
    int parts = std::max(1, std::min(p.nc, (512 + tiles - 1) / tiles));
    c->adj_cgs = (p.nc + parts - 1) / parts;
    c->adj_parts = (p.nc + c->adj_cgs - 1) / c->adj_cgs;
  }
  c->adj_qr = !c->fp64 && (p.ny == 64 || p.ny == 128 || p.ny == 256);
  c->grad_parts = c->adj_qr ? 1 : c->adj_parts;
  c->qr_nblk = std::max(1, std::min(256, c->n / 256));
  c->qr_rows = ((long)c->n + c->qr_nblk - 1) / c->qr_nblk;
  c->qr_rows = (c->qr_rows + 127) / 128 * 128;
  c->qr_nblk = (int)((c->n + c->qr_rows - 1) / c->qr_rows);
  {  // general masks: frames per pass of the operator's per-coil k-space images,
     // as many as fit 256 MiB (at least 16): fewer, larger launches
    const double per_frame = 8.0 * p.nc * (double)c->n;
    c->kc = std::min(p.q, std::max(16, (int)std::min(1e9, (256.0 * 1024 * 1024) / per_frame)));
  }
  carve(c);
  *out = c;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_workspace_bytes(const altgdmin_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ALTGDMIN_EINVAL;
  *bytes = c->bytes;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_set_problem(altgdmin_ctx* c, const void* d_coils, const int32_t* d_mask,
                                     const int32_t* d_m_k, const void* d_y, void* d_ws, void* stream) {
  if (!c || !d_coils || !d_mask || !d_m_k || !d_ws) return ALTGDMIN_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return ALTGDMIN_EINVAL;
  const altgdmin_params& p = c->p;
  c->coils = static_cast<const float2*>(d_coils);
  c->mask = d_mask;
  c->m_k = d_m_k;
  c->y = static_cast<const float2*>(d_y);
  c->ws = static_cast<char*>(d_ws);
  c->stream = static_cast<hipStream_t>(stream);
  c->bound = 0;
  c->initialized = 0;
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, c->st(), 1);
  hipLaunchKernelGGL(k_twiddle, dim3((p.nx + 255) / 256), dim3(256), 0, s, c->at<float2>(c->o_twx), p.nx);
  hipLaunchKernelGGL(k_twiddle, dim3((p.ny + 255) / 256), dim3(256), 0, s, c->at<float2>(c->o_twy), p.ny);
  hipLaunchKernelGGL(k_coil_block, dim3(1024), dim3(256), 0, s, c->coils, c->at<float2>(c->o_coilb), p.nx, p.ny,
                     c->txx, c->n, p.nc);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(c->at<uint32_t>(c->o_bitmap), 0, sizeof(uint32_t) * (size_t)c->n_loc * c->nw, s));
  hipLaunchKernelGGL(k_inv_bitmap, dim3((c->width + 255) / 256, p.q), dim3(256), 0, s, c->mask, c->m_k,
                     c->width, c->per, c->n_loc, c->at<uint32_t>(c->o_bitmap), c->nw, c->st());
  hipLaunchKernelGGL(k_inv_scan, dim3(1), dim3(1024), 0, s, c->at<uint32_t>(c->o_bitmap), c->nw, c->n_loc,
                     c->at<int32_t>(c->o_locptr), c->at<int32_t>(c->o_loc2unit), c->at<int32_t>(c->o_unitloc),
                     c->at<int2>(c->o_unitspan), c->st());
  if (c->lines)
    HIPCHK(launch_gram_work(c->at<int2>(c->o_unitspan), c->at<int4>(c->o_gwork), c->at<int4>(c->o_lineord),
                            c->n_loc, c->st(), s));

  hipLaunchKernelGGL(k_inv_fill, dim3((c->width + 255) / 256, p.q), dim3(256), 0, s, c->mask, c->m_k,
                     c->width, c->per, c->at<uint32_t>(c->o_bitmap), c->nw, c->at<int32_t>(c->o_locptr),
                     c->at<int32_t>(c->o_loc2unit), c->at<int2>(c->o_pairs), c->at<int32_t>(c->o_pairof),
                     c->at<int32_t>(c->o_unitof), c->st());
  HIPCHK(hipGetLastError());
  if (c->y) {
    hipLaunchKernelGGL(k_ysq, dim3(p.q, p.nc), dim3(AG_NT), 0, s, c->y, c->m_k, p.nc, p.m_max,
                       c->at<double>(c->o_ysqp));
    hipLaunchKernelGGL(k_ysq_sum, dim3(1), dim3(128), 0, s, c->at<double>(c->o_ysqp), p.q, p.nc,
                       c->at<double>(c->o_ysq));
    hipLaunchKernelGGL(k_init_stats, dim3(1), dim3(1), 0, s, c->at<double>(c->o_ysq), c->m_k, p.q, p.trunc_c,
                       c->st());
    HIPCHK(hipGetLastError());
    if (c->lines) {
      RowArgs ra{};
      ra.src = c->y;
      ra.dst = c->at<float2>(c->o_T);  // frame-major hybrid data, temporary
      ra.tw = c->at<float2>(c->o_twx);
      ra.nrows = (long)p.q * p.nc * c->lmax;
      ra.m_k = c->m_k;
      ra.nc = p.nc;
      ra.lmax = c->lmax;
      ra.scale = (float)(1.0 / sqrt((double)p.nx));
      ra.st = c->st();
      HIPCHK(launch_rows(p.nx, ra, true, s));
      // per-line layout: the largest pair count is q per line
      hipLaunchKernelGGL(k_build_yu, dim3(p.q * c->width, p.nc), dim3(256), 0, s, c->at<float2>(c->o_T),
                         c->at<int2>(c->o_pairs), c->mask, c->at<int32_t>(c->o_locptr), c->n_loc, c->width,
                         p.nc, p.nx,
                         c->lmax, c->at<float2>(c->o_yh), c->st());
      hipLaunchKernelGGL(k_build_yg, dim3((unsigned)gram_items_bound(c), p.nc), dim3(256), 0, s,
                         c->at<float2>(c->o_yh), c->at<int4>(c->o_gwork), p.nc, p.nx, c->at<float2>(c->o_yg),
                         c->st());
      HIPCHK(hipGetLastError());
    }
  }
  c->bound = 1;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_init(altgdmin_ctx* c, void* d_U) {
  if (!c || !d_U || c->p.r > c->p.q) return ALTGDMIN_EINVAL;  // top r of q singular vectors
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  float2* U = static_cast<float2*>(d_U);
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, c->st(), 0);
  HIPCHK(ag_host::spectral_eig(c, p.r, nullptr));
  float2* X0 = c->at<float2>(c->o_T);
  HIPCHK(launch_x_times_v(X0, c->at<float2>(c->o_Vs), c->n, p.q, p.r, U, c->st(), s));
  // X0 V Sigma^-1 is orthonormal up to FP32 rounding (errors grow with
  // sigma_1 / sigma_r): one CholeskyQR pass restores it
  HIPCHK(cholqr(c, U));
  c->initialized = 1;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_init_from(altgdmin_ctx* c, const void* d_U0, void* d_U) {
  if (!c || !d_U0 || !d_U) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, c->st(), 0);
  if (d_U0 != d_U)
    hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, static_cast<const float2*>(d_U0),
                       static_cast<float2*>(d_U), (long)c->n * p.r);
  HIPCHK(hipGetLastError());
  HIPCHK(cholqr(c, static_cast<float2*>(d_U)));
  HIPCHK(cholqr(c, static_cast<float2*>(d_U)));
  c->initialized = 1;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_cnn_input(altgdmin_ctx* c, float* d_in) {
  if (!c || !d_in) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  float2* X = c->at<float2>(c->o_T);
  HIPCHK(ag_host::adjoint_op(c, c->y, X, 0, 0));
  HIPCHK(launch_cnn_planes(X, c->n, p.q, c->at<double>(c->o_planes), d_in, c->stream));
  return ALTGDMIN_OK;
}

// the learned guess d_M against the fallback basis already in d_U: the step
// size at the fallback, the cost of each, the lower-cost one into d_U
static altgdmin_status warm_combine(altgdmin_ctx* c, const void* d_M, void* d_U, int32_t* d_choice) {
  const altgdmin_params& p = c->p;
  hipStream_t s = c->stream;
  // the step size of Algorithm 2 (first-iteration rule) at the spectral basis:
  // a good learned basis has a much smaller first gradient, and the rule
  // evaluated there would overshoot
  HIPCHK(to_pixmajor(c, static_cast<const float2*>(d_U)));
  HIPCHK(gradient_pieces(c, 0));
  HIPCHK(qr_step_small(c, 2, 0));
  // the gradient pass's solve left the spectral basis's per-frame costs:
  // their sum is the spectral side of the comparison below
  double* f = c->at<double>(c->o_fcmp);
  hipLaunchKernelGGL(k_cost_total, dim3(1), dim3(1), 0, s, c->at<double>(c->o_cost), p.q, f, c->st());
  // an error raised from here on comes from scoring the guess alone
  int32_t* snap = reinterpret_cast<int32_t*>(f + 2);
  hipLaunchKernelGGL(k_err_snapshot, dim3(1), dim3(1), 0, s, c->st(), snap);
  float2* Uc = c->at<float2>(c->o_Uc);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, static_cast<const float2*>(d_M), Uc, (long)c->n * p.r);
  HIPCHK(hipGetLastError());
  HIPCHK(cholqr(c, Uc));
  HIPCHK(cholqr(c, Uc));
  HIPCHK(to_pixmajor(c, Uc));
  HIPCHK(fwd_transform(c, 0));
  HIPCHK(gram_solve(c, 0));
  hipLaunchKernelGGL(k_cost_total, dim3(1), dim3(1), 0, s, c->at<double>(c->o_cost), p.q, f + 1, c->st());
  hipLaunchKernelGGL(k_pick_init, dim3(256), dim3(256), 0, s, f, snap, Uc, static_cast<float2*>(d_U),
                     (long)c->n * p.r, d_choice, c->st());
  hipLaunchKernelGGL(k_err_restore, dim3(1), dim3(1), 0, s, snap, c->st());
  HIPCHK(hipGetLastError());
  c->initialized = 1;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_init_warm(altgdmin_ctx* c, const void* d_M, void* d_U, int32_t* d_choice) {
  if (!c || !d_M || !d_U) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_status st = altgdmin_init(c, d_U);
  if (st != ALTGDMIN_OK) return st;
  return warm_combine(c, d_M, d_U, d_choice);
}

altgdmin_status altgdmin_init_warm_from(altgdmin_ctx* c, const void* d_M, const void* d_Ufb, void* d_U,
                                        int32_t* d_choice) {
  if (!c || !d_M || !d_Ufb || !d_U) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, c->stream, c->st(), 0);
  if (d_Ufb != d_U)
    hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, c->stream, static_cast<const float2*>(d_Ufb),
                       static_cast<float2*>(d_U), (long)c->n * c->p.r);
  HIPCHK(hipGetLastError());
  return warm_combine(c, d_M, d_U, d_choice);
}

altgdmin_status altgdmin_iterate(altgdmin_ctx* c, int32_t n_iter, void* d_U, void* d_B, void* d_U_prev,
                                 int32_t* h_iters_done) {
  if (!c || !d_U) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y || !c->initialized) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  if (n_iter <= 0) n_iter = p.t_max;
  int32_t t0 = 0;
  if (h_iters_done) {
    // the count before this call's iterations: earlier work on the stream first
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&t0, &c->st()->t, sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  HIPCHK(to_pixmajor(c, static_cast<const float2*>(d_U)));
  // every solve also writes B to the caller's buffer (no copy launch after
  // the loop; a halt part-way leaves there the last B computed)
  struct CallScope {  // the caller's buffer is forgotten on every way out
    altgdmin_ctx* c;
    ~CallScope() { c->b_out = nullptr; }
  } scope{c};
  c->b_out = static_cast<float2*>(d_B);
  for (int t = 0; t < n_iter; ++t)
    HIPCHK(one_iteration(c, static_cast<float2*>(d_U), static_cast<float2*>(d_U_prev)));
  if (h_iters_done) {
    int32_t t1 = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&t1, &c->st()->t, sizeof(int32_t), hipMemcpyDeviceToHost));
    *h_iters_done = t1 - t0;
    int32_t err = 0;
    HIPCHK(hipMemcpy(&err, &c->st()->err, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (err) return (altgdmin_status)err;
  }
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_get_eta(altgdmin_ctx* c, double* eta) {
  if (!c || !eta) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(eta, &c->st()->eta, sizeof(double), hipMemcpyDeviceToHost));
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_set_eta(altgdmin_ctx* c, double eta) {
  if (!c || !isfinite(eta)) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  hipLaunchKernelGGL(k_state_set_eta, dim3(1), dim3(1), 0, c->stream, c->st(), eta > 0 ? eta : -1.0);
  return map_hip(hipGetLastError());
}

altgdmin_status altgdmin_cost(altgdmin_ctx* c, const void* d_U, double* d_f) {
  if (!c || !d_U || !d_f) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  // the last iteration's statistics read cost_k, which the solve below overwrites
  HIPCHK(launch_stats_finish(c->st(), c->at<double2>(c->o_stsrc), c->at<double>(c->o_cost), c->p.q, c->p.r,
                             c->stream));
  HIPCHK(to_pixmajor(c, static_cast<const float2*>(d_U)));
  HIPCHK(fwd_transform(c, 0));
  HIPCHK(gram_solve(c, 0));
  hipLaunchKernelGGL(k_cost_total, dim3(1), dim3(1), 0, c->stream, c->at<double>(c->o_cost), c->p.q, d_f,
                     c->st());
  return map_hip(hipGetLastError());
}

altgdmin_status altgdmin_gradient(altgdmin_ctx* c, const void* d_U, void* d_B, void* d_G) {
  if (!c || !d_U) return ALTGDMIN_EINVAL;
  if (!c->bound || !c->y) return ALTGDMIN_ESTATE;
  const altgdmin_params& p = c->p;
  HIPCHK(launch_stats_finish(c->st(), c->at<double2>(c->o_stsrc), c->at<double>(c->o_cost), p.q, p.r, c->stream));
  HIPCHK(to_pixmajor(c, static_cast<const float2*>(d_U)));
  if (!d_G) {  // the LS step alone
    HIPCHK(fwd_transform(c, 0));
    HIPCHK(gram_solve(c, 0));
    if (d_B)
      hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, c->stream, c->at<float2>(c->o_B), static_cast<float2*>(d_B),
                         (long)p.q * p.r);
    return map_hip(hipGetLastError());
  }
  HIPCHK(gradient_pieces(c, 0));
  if (c->grad_parts > 1)
    hipLaunchKernelGGL(k_sum_parts, dim3(1024), dim3(256), 0, c->stream, c->at<float2>(c->o_G),
                       (long)c->n * p.r, c->grad_parts, c->at<float2>(c->o_G), (long)c->n * p.r);
  if (d_B)
    hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, c->stream, c->at<float2>(c->o_B),
                       static_cast<float2*>(d_B), (long)p.q * p.r);
  if (d_G)
    hipLaunchKernelGGL(k_to_colmajor, dim3(1024), dim3(256), 0, c->stream, c->at<float2>(c->o_G), p.r,
                       (long)c->n, static_cast<float2*>(d_G));
  return map_hip(hipGetLastError());
}

altgdmin_status altgdmin_apply_A(altgdmin_ctx* c, const void* d_X, void* d_Y) {
  if (!c || !d_X || !d_Y) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  return map_hip(ag_host::forward_op(c, static_cast<const float2*>(d_X), static_cast<float2*>(d_Y)));
}

altgdmin_status altgdmin_apply_AH(altgdmin_ctx* c, const void* d_Y, void* d_X) {
  if (!c || !d_X || !d_Y) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  return map_hip(ag_host::adjoint_op(c, static_cast<const float2*>(d_Y), static_cast<float2*>(d_X), 0, 0));
}

altgdmin_status altgdmin_get_stats(altgdmin_ctx* c, altgdmin_stats* out) {
  if (!c || !out) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  DevState h;
  HIPCHK(launch_stats_finish(c->st(), c->at<double2>(c->o_stsrc), c->at<double>(c->o_cost), c->p.q, c->p.r,
                             c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(&h, c->st(), sizeof(DevState), hipMemcpyDeviceToHost));
  out->t = h.t;
  out->exited = h.exited;
  out->f = h.f;
  out->sd = h.sd;
  out->grad_norm = h.grad_norm;
  out->eta = h.eta;
  out->gamma = h.gamma;
  out->n_trunc = h.n_trunc;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_last_error(altgdmin_ctx* c, int32_t* frame) {
  if (!c) return ALTGDMIN_EINVAL;
  if (!c->bound) return ALTGDMIN_ESTATE;
  int32_t v[2];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(v, c->st(), sizeof(v), hipMemcpyDeviceToHost));
  if (frame) *frame = v[0] ? v[1] : -1;
  if (v[0]) {
    const int32_t z[2] = {0, -1};
    HIPCHK(hipMemcpy(c->st(), z, sizeof(z), hipMemcpyHostToDevice));
  }
  return (altgdmin_status)v[0];
}

altgdmin_status altgdmin_set_timing(altgdmin_ctx* c, int32_t which) {
  if (!c || which < 0 || which >= TK_COUNT) return ALTGDMIN_EINVAL;
  c->timed = which;
  c->ev_used = 0;
  return ALTGDMIN_OK;
}

altgdmin_status altgdmin_kernel_time(altgdmin_ctx* c, const char** name, int32_t* launches, double* total_ms) {
  if (!c) return ALTGDMIN_EINVAL;
  if (name) *name = kTimedNames[c->timed];
  double tot = 0.0;
  int32_t cnt = 0;
  if (c->ev_used >= 2) {
    HIPCHK(hipEventSynchronize(c->ev[c->ev_used - 1]));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
      tot += ms;
      ++cnt;
    }
  }
  c->ev_used = 0;
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = tot;
  return ALTGDMIN_OK;
}

void altgdmin_destroy(altgdmin_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
