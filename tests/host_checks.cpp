// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py).
// Only entry points and paths that make no GPU call are exercised: context
// creation over a grid of shapes (workspace and auxiliary sizes, the
// built-in scratch bound), every parameter check, null arguments and calls
// on a context with no problem bound, and the warm-start network's host
// bookkeeping.  Exits non-zero at the first failed expectation; the
// sanitizers abort on the first error they find.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>

#include "altgdmin.h"
#include "wsinit.h"

static int g_checks = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    ++g_checks;                                                          \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

static altgdmin_params base_params() {
  altgdmin_params p{};
  p.nx = 64;
  p.ny = 64;
  p.nc = 4;
  p.q = 16;
  p.r = 4;
  p.m_max = 1024;
  p.mask_kind = ALTGDMIN_MASK_LINES;
  p.precision = ALTGDMIN_FP32;
  p.trunc_c = 36.0;
  p.eta_c = 0.14;
  p.eta_cap_c = 0.0;
  p.eps_exit = 0.0;
  p.t_max = 70;
  p.exit_consec = 1;
  return p;
}

static void expect_rejected(const altgdmin_params& p) {
  altgdmin_ctx* c = reinterpret_cast<altgdmin_ctx*>(0x1);
  EXPECT(altgdmin_create(&p, &c) == ALTGDMIN_EINVAL);
  EXPECT(c == nullptr);
}

// every call on a context whose problem is not bound: a state error (or an
// argument error) before any GPU work
static void unbound_calls(altgdmin_ctx* c) {
  char buf[256];
  void* d = buf;
  int32_t i32 = 0;
  double f64 = 0.0;
  altgdmin_stats st{};
  EXPECT(altgdmin_init(c, d) != ALTGDMIN_OK);
  EXPECT(altgdmin_init_from(c, d, d) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_cnn_input(c, reinterpret_cast<float*>(d)) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_init_warm(c, d, d, &i32) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_init_warm_from(c, d, d, d, &i32) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_iterate(c, 1, d, d, d, &i32) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_get_eta(c, &f64) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_set_eta(c, 0.1) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_cost(c, d, &f64) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_gradient(c, d, d, d) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_apply_A(c, d, d) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_apply_AH(c, d, d) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_get_stats(c, &st) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_last_error(c, &i32) == ALTGDMIN_ESTATE);
  // the auxiliary workspace must be 256-byte aligned: a misaligned one is an
  // argument error, an aligned one a state error
  alignas(256) static char aux[512];
  EXPECT(altgdmin_mean(c, 1e-3, 10, d, aux + 1, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_mean(c, 1e-3, 10, d, aux, &i32) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_residual(c, d, nullptr, d, aux) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_mec_cgls(c, d, 3, 0.0, d, aux) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_mec_ista(c, d, 10, 1e-3, 0.0025, d, aux, &i32) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_expand(c, d, d, nullptr, nullptr, d) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_rank_energy(c, 1, &f64, aux) == ALTGDMIN_ESTATE);
  EXPECT(altgdmin_auto_rank(c, 85.0, &i32, &i32, aux) == ALTGDMIN_ESTATE);
  // argument errors come first
  EXPECT(altgdmin_mean(c, -1.0, 10, d, aux, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_mean(c, NAN, 10, d, aux, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_mean(c, 1e-3, -1, d, aux, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_mec_ista(c, d, -1, 1e-3, 0.0025, d, aux, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_expand(c, d, nullptr, nullptr, nullptr, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_rank_energy(c, 0, &f64, aux) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_rank_energy(c, 17, &f64, aux) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_auto_rank(c, 0.0, &i32, &i32, aux) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_auto_rank(c, 100.5, &i32, &i32, aux) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_set_eta(c, INFINITY) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_set_problem(c, d, reinterpret_cast<int32_t*>(d), reinterpret_cast<int32_t*>(d), d,
                              static_cast<char*>(static_cast<void*>(aux)) + 8, nullptr) == ALTGDMIN_EINVAL);
  // timing bookkeeping without events
  EXPECT(altgdmin_set_timing(c, -1) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_set_timing(c, 3) == ALTGDMIN_OK);
  const char* name = nullptr;
  double ms = -1.0;
  EXPECT(altgdmin_kernel_time(c, &name, &i32, &ms) == ALTGDMIN_OK);
  EXPECT(name != nullptr && i32 == 0 && ms == 0.0);
  EXPECT(altgdmin_set_timing(c, 0) == ALTGDMIN_OK);
}

static void null_context_calls() {
  char buf[64];
  void* d = buf;
  int32_t i32 = 0;
  double f64 = 0.0;
  size_t sz = 0;
  altgdmin_stats st{};
  altgdmin_params p = base_params();
  EXPECT(altgdmin_create(&p, nullptr) == ALTGDMIN_EINVAL);
  altgdmin_ctx* c = nullptr;
  EXPECT(altgdmin_create(nullptr, &c) == ALTGDMIN_EINVAL && c == nullptr);
  EXPECT(altgdmin_workspace_bytes(nullptr, &sz) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_aux_bytes(nullptr, &sz) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_set_problem(nullptr, d, nullptr, nullptr, d, d, nullptr) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_init(nullptr, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_init_from(nullptr, d, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_iterate(nullptr, 1, d, d, d, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_get_eta(nullptr, &f64) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_cost(nullptr, d, &f64) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_gradient(nullptr, d, d, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_apply_A(nullptr, d, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_apply_AH(nullptr, d, d) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_get_stats(nullptr, &st) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_last_error(nullptr, &i32) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_kernel_time(nullptr, nullptr, nullptr, nullptr) == ALTGDMIN_EINVAL);
  EXPECT(altgdmin_mean_noalloc(nullptr, 1e-3, 10, d, &i32) == ALTGDMIN_EINVAL);
  altgdmin_destroy(nullptr);
  for (int s = ALTGDMIN_OK; s <= ALTGDMIN_ESCRATCH; ++s)
    EXPECT(altgdmin_status_string(static_cast<altgdmin_status>(s)) != nullptr);
}

static void parameter_checks() {
  altgdmin_params p = base_params();
  altgdmin_params b;
  b = p; b.nx = 48; expect_rejected(b);
  b = p; b.ny = 4; expect_rejected(b);
  b = p; b.nx = 1024; expect_rejected(b);
  b = p; b.nc = 0; expect_rejected(b);
  b = p; b.nc = 65; expect_rejected(b);
  b = p; b.q = 0; expect_rejected(b);
  b = p; b.q = 129; expect_rejected(b);
  b = p; b.r = 0; expect_rejected(b);
  b = p; b.r = 17; expect_rejected(b);
  b = p; b.mask_kind = 7; expect_rejected(b);
  b = p; b.precision = 9; expect_rejected(b);
  b = p; b.m_max = 0; expect_rejected(b);
  b = p; b.m_max = p.nx * p.ny + 1; expect_rejected(b);
  b = p; b.m_max = 1000; expect_rejected(b);  // LINES: whole lines only
  b = p; b.eta_c = 0.0; expect_rejected(b);
  b = p; b.eta_c = NAN; expect_rejected(b);
  b = p; b.trunc_c = INFINITY; expect_rejected(b);
  b = p; b.eta_cap_c = -1.0; expect_rejected(b);
  b = p; b.eps_exit = NAN; expect_rejected(b);
  b = p; b.exit_consec = -1; expect_rejected(b);
  b = p; b.t_max = 0; expect_rejected(b);
}

// creation over a grid of shapes: the size arithmetic of the workspace
// carve, the auxiliary workspace and the scratch bound
static void shape_grid() {
  const int sizes[] = {8, 64, 256, 512};
  const int coils[] = {1, 12, 64};
  const int frames[] = {1, 40, 128};
  const int ranks[] = {1, 8, 16};
  int made = 0;
  for (int nx : sizes)
    for (int ny : sizes)
      for (int nc : coils)
        for (int q : frames)
          for (int r : ranks)
            for (int kind = 0; kind < 2; ++kind)
              for (int prec = 0; prec < 2; ++prec) {
                altgdmin_params p = base_params();
                p.nx = nx;
                p.ny = ny;
                p.nc = nc;
                p.q = q;
                p.r = r;
                p.mask_kind = kind == 0 ? ALTGDMIN_MASK_LINES : ALTGDMIN_MASK_INDEX;
                p.precision = prec == 0 ? ALTGDMIN_FP32 : ALTGDMIN_MIXED;
                p.m_max = kind == 0 ? nx * std::max(1, ny / 8) : std::max(1, nx * ny / 8);
                altgdmin_ctx* c = nullptr;
                const altgdmin_status s = altgdmin_create(&p, &c);
                EXPECT(s == ALTGDMIN_OK);
                size_t ws = 0, aux = 0;
                EXPECT(altgdmin_workspace_bytes(c, &ws) == ALTGDMIN_OK);
                EXPECT(altgdmin_aux_bytes(c, &aux) == ALTGDMIN_OK);
                EXPECT(ws > 0 && ws % 256 == 0 && aux > 0);
                // W and K alone: two planes of nc r complex values per image row kept
                const size_t wk = 2ull * 8ull * nc * r * (size_t)ny * nx;
                EXPECT(ws >= wk);
                int32_t it = 0;
                char z[16];
                const altgdmin_status sm = altgdmin_mean_noalloc(c, 1e-3, 10, z, &it);
                EXPECT(sm == ALTGDMIN_ESCRATCH || sm == ALTGDMIN_ESTATE);
                if (made % 97 == 0) unbound_calls(c);
                altgdmin_destroy(c);
                ++made;
              }
  EXPECT(made == 4 * 4 * 3 * 3 * 3 * 2 * 2);
}

static void warm_start_network() {
  wsinit_ctx* h = nullptr;
  EXPECT(wsinit_create(64, 64, 16, 4, 32, 4, 2, nullptr, nullptr) == ALTGDMIN_EINVAL);
  EXPECT(wsinit_create(60, 64, 16, 4, 32, 4, 2, nullptr, &h) == ALTGDMIN_EINVAL && h == nullptr);
  EXPECT(wsinit_create(64, 64, 16, 4, 32, 3, 2, nullptr, &h) == ALTGDMIN_EINVAL);
  EXPECT(wsinit_create(64, 64, 16, 4, 33, 4, 2, nullptr, &h) == ALTGDMIN_EINVAL);
  EXPECT(wsinit_create(64, 64, 16, 4, 32, 4, 65, nullptr, &h) == ALTGDMIN_EINVAL);
  const int dims[][4] = {{64, 64, 16, 4}, {256, 256, 40, 8}, {128, 128, 100, 10}, {8, 512, 1, 16}};
  for (const auto& dm : dims)
    for (int width : {4, 32})
      for (int batch : {1, 8}) {
        EXPECT(wsinit_create(dm[0], dm[1], dm[2], dm[3], width, 4, batch, nullptr, &h) == ALTGDMIN_OK);
        int64_t np = 0;
        size_t ws = 0;
        EXPECT(wsinit_param_count(h, &np) == ALTGDMIN_OK);
        // conv 3x3: 2q -> w -> w -> w -> 2r, each with biases
        const int64_t want = (int64_t)width * 2 * dm[2] * 9 + width + 2 * ((int64_t)width * width * 9 + width) +
                             (int64_t)2 * dm[3] * width * 9 + 2 * dm[3];
        EXPECT(np == want);
        EXPECT(wsinit_workspace_bytes(h, &ws) == ALTGDMIN_OK && ws > 0);
        float f = 0.f;
        double dl = 0.0;
        char w[16];
        EXPECT(wsinit_forward(h, &f, &f, 0, w, w) == ALTGDMIN_EINVAL);
        EXPECT(wsinit_forward(h, &f, &f, batch + 1, w, w) == ALTGDMIN_EINVAL);
        EXPECT(wsinit_loss_backward(h, &f, &f, w, 1, &f, &dl, nullptr) == ALTGDMIN_EINVAL);
        EXPECT(wsinit_adam_step(h, &f, &f, &f, &f, 1e-3f, 0) == ALTGDMIN_EINVAL);
        EXPECT(wsinit_adam_step(h, &f, &f, &f, &f, 0.f, 1) == ALTGDMIN_EINVAL);
        wsinit_destroy(h);
      }
  EXPECT(wsinit_param_count(nullptr, nullptr) == ALTGDMIN_EINVAL);
  wsinit_destroy(nullptr);
}

int main() {
  null_context_calls();
  parameter_checks();
  shape_grid();
  warm_start_network();
  std::printf("host checks passed: %d\n", g_checks);
  return 0;
}
